// Host runtime and C-ABI of the batched form (include/mcinv.h, mcinv_batch_*).
//
// All matrices are prepared exactly like a single-matrix context (prep.h) and
// concatenated: global positions, entries pointing at global positions,
// matrix m's noise stream = m.  One sweep is described once as a list of
// work items in (colour, matrix, chunk) order; a launch runs that list
// nsweeps times in one persistent kernel (batch.hip).  Each (sweeps, sample)
// launch shape is captured once into a HIP graph and replayed: its arguments
// never change, the kernel reads the current sweep and sample counts from a
// device-resident clock it advances itself.  The autotuner times candidate
// (rows per work item, items per queue access) pairs on burn-in sweeps.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <string>
#include <utility>
#include <vector>

#include "../../include/mcinv.h"
#include "boundary.h"
#include "batch.h"
#include "device_common.h"
#include "prep.h"
#include "moments.h"
#include "sweep.h"

using namespace mcinv;

namespace {

thread_local std::string g_berror;
constexpr int32_t kBlockSlots = 16;      // time batches of the block accumulator
constexpr int32_t kDiagSlotsSmallG = 16; // time batches of the diagonal when G < 16
constexpr int64_t kMaxItemsPerLaunch = (int64_t)1 << 30;

}  // namespace

struct mcinv_batch {
    mcinv_batch_config cfg{};
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int64_t M = 0;
    int32_t P = 64, G = 16, lane_shift = 4;
    std::vector<Prepared> prep;
    std::vector<bool> loaded;
    bool committed = false;
    std::vector<int64_t> row0;
    int64_t nrows = 0, nnz_total = 0;
    int32_t max_colors = 0;

    RowRec* d_rows = nullptr;
    Entry<float>* d_ent = nullptr;
    Scales<float>* d_sc = nullptr;
    float* d_z = nullptr;
    float* d_w = nullptr;
    BMat* d_mats = nullptr;
    uint32_t* d_done = nullptr;
    BatchClock* d_clock = nullptr;
    int32_t* d_flag = nullptr;
    int64_t* d_orig = nullptr;   // global position -> row0 + original row

    // schedule
    int32_t rows_per_item = 64, grab = 4, grid = 0;
    BItem* d_items_burn = nullptr;
    BItem* d_items_sample = nullptr;
    BMat* d_mats_sample = nullptr;
    size_t cap_items_burn = 0, cap_items_sample = 0, cap_mats_burn = 0, cap_mats_sample = 0;  // allocated lengths
    int64_t ips_burn = 0, ips_sample = 0;
    int32_t schedule = MCINV_SCHEDULE_PHASED;
    // phase boundaries of the item lists (burn, sample) and whether a phase is
    // the block-moment phase
    std::vector<int64_t> phase_off[2];
    std::vector<bool> phase_block[2];
    std::map<std::pair<int64_t, int>, std::pair<hipGraph_t, hipGraphExec_t>> graphs;

    // moments
    uint32_t flags = 0;
    bool requested = false;
    int32_t bdim = 0;
    std::vector<int64_t> hI, hJ;   // [M][bdim] global positions
    int64_t* d_bI = nullptr;
    int64_t* d_bJ = nullptr;
    double* d_diag = nullptr;
    double* d_block = nullptr;
    int32_t nslots_diag = 1;
    int64_t batch_len = 1;
    int64_t samples = 0, sweeps = 0;
    double* d_slot_len = nullptr;
    double* d_est = nullptr;
    double* d_se = nullptr;
    double last_ms = 0.0;

    // Per-matrix stopping (mcinv_batch_sample_until_each): a matrix that met
    // the tolerance is left out of the item lists, so its chains and
    // accumulators stay as they were when it stopped.
    std::vector<uint8_t> active;
    std::vector<int64_t> msamples;          // samples accumulated per matrix
    std::vector<double> mrel;               // per matrix: max se/|est| at its last check
    int32_t* d_row_mat = nullptr;           // position -> matrix
    int64_t* d_row0 = nullptr;              // [M + 1] first position of each matrix
    double* d_rel = nullptr;                // [nrows] se/|est| per position at the last check
    double* d_mrel = nullptr;               // [M] per-matrix max of d_rel

    std::string err;
};

namespace {

mcinv_status bfail(mcinv_batch* b, mcinv_status code, const std::string& msg)
{
    if (b)
        b->err = msg;
    else
        g_berror = msg;
    return code;
}

#define BHIP(b, expr)                                                                           \
    do {                                                                                        \
        hipError_t e_ = (expr);                                                                 \
        if (e_ != hipSuccess)                                                                   \
            return bfail((b), e_ == hipErrorOutOfMemory ? MCINV_ENOMEM : MCINV_EDEVICE,         \
                         std::string(#expr) + ": " + hipGetErrorString(e_));                    \
    } while (0)

#define BTRY(expr)                      \
    do {                                \
        mcinv_status s_ = (expr);       \
        if (s_ != MCINV_OK) return s_;  \
    } while (0)

template <typename T>
void bfree(T*& p)
{
    if (p) (void)hipFree((void*)p);
    p = nullptr;
}

template <typename T>
mcinv_status balloc(mcinv_batch* b, T** p, size_t count)
{
    *p = nullptr;
    BHIP(b, hipMalloc((void**)p, std::max<size_t>(count, 1) * sizeof(T)));
    return MCINV_OK;
}

template <typename T>
mcinv_status bupload(mcinv_batch* b, T** p, const std::vector<T>& h)
{
    bfree(*p);
    BTRY(balloc(b, p, h.size()));
    if (!h.empty()) BHIP(b, hipMemcpyAsync(*p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, b->stream));
    return MCINV_OK;
}

// Upload into a device array that is reallocated only when it must grow.
template <typename T>
mcinv_status bupload_keep(mcinv_batch* b, T** p, size_t* cap, const std::vector<T>& h)
{
    if (*p == nullptr || h.size() > *cap) {
        bfree(*p);
        BTRY(balloc(b, p, h.size()));
        *cap = std::max<size_t>(h.size(), 1);
    }
    if (!h.empty()) BHIP(b, hipMemcpyAsync(*p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, b->stream));
    return MCINV_OK;
}

void drop_graphs(mcinv_batch* b)
{
    for (auto& kv : b->graphs) {
        (void)hipGraphExecDestroy(kv.second.second);
        (void)hipGraphDestroy(kv.second.first);
    }
    b->graphs.clear();
}

// One sweep's items: colours ascending, matrices ascending, chunks of
// rows_per_item rows; then (sampling with a block) one block item per matrix.
// Matrices that have stopped (not active) get no items.
mcinv_status build_items(mcinv_batch* b)
{
    for (int pass = 0; pass < 2; ++pass) {
        const bool with_block = pass == 1 && b->bdim > 0 && (b->flags & MCINV_REQ_BLOCK);
        std::vector<BItem> items;
        std::vector<int32_t> per_m(b->M, 0);
        b->phase_off[pass].clear();
        b->phase_block[pass].clear();
        for (int32_t c = 0; c < b->max_colors; ++c) {
            b->phase_off[pass].push_back((int64_t)items.size());
            b->phase_block[pass].push_back(false);
            for (int64_t m = 0; m < b->M; ++m) {
                const Prepared& h = b->prep[m];
                if (c >= h.ncolors || !b->active[m]) continue;
                const int64_t beg = b->row0[m] + h.color_ptr[c], end = b->row0[m] + h.color_ptr[c + 1];
                const int32_t prior = per_m[m];
                for (int64_t r = beg; r < end; r += b->rows_per_item) {
                    BItem it{};
                    it.m = (int32_t)m;
                    it.kind = 0;
                    it.row_begin = r;
                    it.row_end = std::min<int64_t>(end, r + b->rows_per_item);
                    it.prior = prior;
                    items.push_back(it);
                    per_m[m]++;
                }
            }
        }
        if (with_block) {
            b->phase_off[pass].push_back((int64_t)items.size());
            b->phase_block[pass].push_back(true);
        }
        if (with_block)
            for (int64_t m = 0; m < b->M; ++m) {
                if (!b->active[m]) continue;
                BItem it{};
                it.m = (int32_t)m;
                it.kind = 1;
                it.prior = per_m[m];
                items.push_back(it);
                per_m[m]++;
            }
        b->phase_off[pass].push_back((int64_t)items.size());
        std::vector<BMat> mats(b->M);
        for (int64_t m = 0; m < b->M; ++m) {
            mats[m].row0 = b->row0[m];
            mats[m].n = b->prep[m].n;
            mats[m].items_per_sweep = per_m[m];
            mats[m].stream = (uint32_t)m;
            mats[m].blk = b->bdim > 0 ? m * b->bdim : -1;
        }
        if (pass == 0) {
            BTRY(bupload_keep(b, &b->d_items_burn, &b->cap_items_burn, items));
            BTRY(bupload_keep(b, &b->d_mats, &b->cap_mats_burn, mats));
            b->ips_burn = (int64_t)items.size();
        } else {
            BTRY(bupload_keep(b, &b->d_items_sample, &b->cap_items_sample, items));
            BTRY(bupload_keep(b, &b->d_mats_sample, &b->cap_mats_sample, mats));
            b->ips_sample = (int64_t)items.size();
        }
    }
    BHIP(b, hipStreamSynchronize(b->stream));
    drop_graphs(b);
    return MCINV_OK;
}

mcinv_status commit(mcinv_batch* b)
{
    if (b->committed) return MCINV_OK;
    for (int64_t m = 0; m < b->M; ++m)
        if (!b->loaded[m]) return bfail(b, MCINV_ESTATE, "matrix " + std::to_string(m) + " was not loaded");
    b->row0.assign(b->M + 1, 0);
    int64_t ents = 0;
    for (int64_t m = 0; m < b->M; ++m) {
        b->row0[m + 1] = b->row0[m] + b->prep[m].n;
        ents += (int64_t)b->prep[m].ent.size();
        b->max_colors = std::max(b->max_colors, b->prep[m].ncolors);
        b->nnz_total += b->prep[m].nnz;
    }
    b->nrows = b->row0[b->M];
    if (b->nrows > INT32_MAX) return bfail(b, MCINV_EINVAL, "too many rows in the batch");
    std::vector<RowRec> rows(b->nrows);
    std::vector<Entry<float>> ent;
    ent.reserve(ents);
    std::vector<Scales<float>> sc(b->nrows);
    std::vector<int64_t> orig(b->nrows);
    for (int64_t m = 0; m < b->M; ++m) {
        const Prepared& h = b->prep[m];
        const int64_t r0 = b->row0[m];
        for (int64_t q = 0; q < h.n; ++q) {
            RowRec rr = h.rows[q];
            const int64_t first = (int64_t)ent.size();
            for (int64_t e = rr.begin; e < rr.begin + rr.count; ++e) {
                Entry<float> x{};
                x.col = (int32_t)(r0 + h.ent[e].col);
                x.u = cast_val<float>(h.ent[e].u);
                x.v = cast_val<float>(h.ent[e].v);
                ent.push_back(x);
            }
            rr.begin = first;
            rows[r0 + q] = rr;
            sc[r0 + q].a = cast_val<float>(h.a[q]);
            sc[r0 + q].b = cast_val<float>(h.b[q]);
            orig[r0 + q] = r0 + h.perm[q];
        }
    }
    BTRY(bupload(b, &b->d_rows, rows));
    BTRY(bupload(b, &b->d_ent, ent));
    BTRY(bupload(b, &b->d_sc, sc));
    BTRY(bupload(b, &b->d_orig, orig));
    std::vector<int32_t> row_mat(b->nrows);
    for (int64_t m = 0; m < b->M; ++m)
        for (int64_t q = b->row0[m]; q < b->row0[m + 1]; ++q) row_mat[q] = (int32_t)m;
    BTRY(bupload(b, &b->d_row_mat, row_mat));
    BTRY(bupload(b, &b->d_row0, b->row0));
    BTRY(balloc(b, &b->d_rel, (size_t)b->nrows));
    BTRY(balloc(b, &b->d_mrel, (size_t)b->M));
    bfree(b->d_slot_len);
    BTRY(balloc(b, &b->d_slot_len, (size_t)b->M * std::max(kBlockSlots, kDiagSlotsSmallG)));
    b->active.assign(b->M, 1);
    b->msamples.assign(b->M, 0);
    b->mrel.assign(b->M, INFINITY);
    const size_t sbytes = (size_t)b->nrows * b->P * sizeof(float);
    BHIP(b, hipMalloc((void**)&b->d_z, sbytes));
    BHIP(b, hipMalloc((void**)&b->d_w, sbytes));
    BHIP(b, hipMemsetAsync(b->d_z, 0, sbytes, b->stream));
    BHIP(b, hipMemsetAsync(b->d_w, 0, sbytes, b->stream));
    BTRY(balloc(b, &b->d_done, (size_t)b->M));
    BHIP(b, hipMemsetAsync(b->d_done, 0, sizeof(uint32_t) * b->M, b->stream));
    BTRY(build_items(b));
    BHIP(b, hipStreamSynchronize(b->stream));
    b->committed = true;
    return MCINV_OK;
}

BatchArgs make_args(mcinv_batch* b, int64_t nsweeps, bool sample)
{
    BatchArgs a{};
    a.rows = b->d_rows;
    a.ent = b->d_ent;
    a.sc = b->d_sc;
    a.z = b->d_z;
    a.w = b->d_w;
    a.P = b->P;
    a.lane_shift = b->lane_shift;
    a.items = sample ? b->d_items_sample : b->d_items_burn;
    a.items_per_sweep = sample ? b->ips_sample : b->ips_burn;
    a.nsweeps = nsweeps;
    a.sample = sample ? 1 : 0;
    a.grab = b->grab;
    a.mats = sample ? b->d_mats_sample : b->d_mats;
    a.nmats = (int32_t)b->M;
    a.done = b->d_done;
    a.clock = b->d_clock;
    a.key0 = (uint32_t)(b->cfg.seed & 0xffffffffu);
    a.key1 = (uint32_t)(b->cfg.seed >> 32);
    a.noise = b->cfg.noise;
    a.spin_limit = 1u << 24;
    a.G = b->G;
    a.nslots_diag = b->nslots_diag;
    a.nslots_block = kBlockSlots;
    a.batch_len = b->batch_len;
    a.nrows = b->nrows;
    a.diag = sample && (b->flags & MCINV_REQ_DIAG) ? b->d_diag : nullptr;
    a.bdim = b->bdim;
    a.bI = b->d_bI;
    a.bJ = b->d_bJ;
    a.block = sample && (b->flags & MCINV_REQ_BLOCK) ? b->d_block : nullptr;
    a.flag = b->d_flag;
    a.thresh = 1e30f;
    return a;
}

// One call's sweeps on the stream: a single persistent launch, or per sweep
// one launch per phase followed by the clock tick.
hipError_t run_launch(mcinv_batch* b, int64_t nsweeps, bool sample)
{
    const BatchArgs a = make_args(b, nsweeps, sample);
    if (b->schedule == MCINV_SCHEDULE_PERSISTENT) return launch_batch(a, b->grid, b->stream);
    const int pass = sample ? 1 : 0;
    const std::vector<int64_t>& off = b->phase_off[pass];
    for (int64_t k = 0; k < nsweeps; ++k) {
        for (size_t p = 0; p + 1 < off.size(); ++p) {
            const hipError_t e = launch_batch_phase(a, a.items + off[p], off[p + 1] - off[p],
                                                    b->phase_block[pass][p], b->stream);
            if (e != hipSuccess) return e;
        }
        const hipError_t e = launch_batch_tick(b->d_clock, sample, b->stream);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Runs nsweeps sweeps as graph replays of one persistent launch each.
mcinv_status run_sweeps(mcinv_batch* b, int64_t nsweeps, bool sample, bool use_graph = true)
{
    const int64_t ips = sample ? b->ips_sample : b->ips_burn;
    const int64_t per_launch = std::max<int64_t>(1, std::min<int64_t>(nsweeps, kMaxItemsPerLaunch / std::max<int64_t>(ips, 1)));
    int64_t left = nsweeps;
    while (left > 0) {
        const int64_t k = std::min(left, per_launch);
        if (use_graph) {
            auto key = std::make_pair(k, sample ? 1 : 0);
            auto found = b->graphs.find(key);
            if (found == b->graphs.end()) {
                hipGraph_t g = nullptr;
                hipGraphExec_t ge = nullptr;
                BHIP(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
                const hipError_t le = run_launch(b, k, sample);
                const hipError_t ce = hipStreamEndCapture(b->stream, &g);
                BHIP(b, le);
                BHIP(b, ce);
                BHIP(b, hipGraphInstantiate(&ge, g, nullptr, nullptr, 0));
                found = b->graphs.emplace(key, std::make_pair(g, ge)).first;
            }
            BHIP(b, hipGraphLaunch(found->second.second, b->stream));
        } else {
            BHIP(b, run_launch(b, k, sample));
        }
        left -= k;
        b->sweeps += k;
        if (sample) {
            b->samples += k;
            for (int64_t m = 0; m < b->M; ++m)
                if (b->active[m]) b->msamples[m] += k;
        }
    }
    return MCINV_OK;
}

mcinv_status check_after(mcinv_batch* b)
{
    int32_t flag = 0;
    BatchClock clk{};
    BHIP(b, hipMemcpyAsync(&flag, b->d_flag, sizeof(flag), hipMemcpyDeviceToHost, b->stream));
    BHIP(b, hipMemcpyAsync(&clk, b->d_clock, sizeof(clk), hipMemcpyDeviceToHost, b->stream));
    BHIP(b, hipStreamSynchronize(b->stream));
    if (clk.error) return bfail(b, MCINV_EDEVICE, "batched launch: a dependency wait exceeded its bound");
    if (clk.sweep != b->sweeps) return bfail(b, MCINV_EDEVICE, "batched launch: device sweep count disagrees");
    if (flag) return bfail(b, MCINV_EDIVERGED, "chain state became non-finite or exceeded 1e30");
    return MCINV_OK;
}

// With fewer than 16 chain groups the diagonal's error clusters include time
// batches, which must be long against the chains' autocorrelation to be
// independent (the single path accepts a stop only once its batches span 16
// sweeps); here their length is fixed by expected_samples, so a stopping rule
// on shorter batches is refused up front.
constexpr int64_t kMinStopBatchLen = 16;

mcinv_status check_stop_batches(mcinv_batch* b)
{
    if (b->nslots_diag > 1 && b->batch_len < kMinStopBatchLen)
        return bfail(b, MCINV_EINVAL,
                     "with fewer than 16 chain groups the error clusters are time batches of " +
                         std::to_string(b->batch_len) + " sweeps; a stopping rule needs batches of at least " +
                         std::to_string(kMinStopBatchLen) + " (set_requested with expected_samples >= " +
                         std::to_string(kMinStopBatchLen * kBlockSlots) + ")");
    return MCINV_OK;
}

std::vector<double> slot_lengths(int64_t samples, int64_t L, int32_t nslots)
{
    std::vector<double> len(nslots, 0.0);
    for (int32_t s = 0; s < nslots; ++s) {
        const int64_t beg = s * L;
        const int64_t end = (s == nslots - 1) ? samples : std::min(samples, (s + 1) * L);
        len[s] = (double)std::max<int64_t>(0, end - beg);
    }
    return len;
}

// Estimates and SEs of every matrix's diagonal, each over its own samples
// (into d_est / d_se); with want_max only each matrix's max se/|est|, into
// b->mrel.
mcinv_status finalize_diag_all(mcinv_batch* b, bool want_max)
{
    std::vector<double> len((size_t)b->M * b->nslots_diag);
    for (int64_t m = 0; m < b->M; ++m) {
        const std::vector<double> l = slot_lengths(b->msamples[m], b->batch_len, b->nslots_diag);
        std::copy(l.begin(), l.end(), len.begin() + m * b->nslots_diag);
    }
    BHIP(b, hipMemcpyAsync(b->d_slot_len, len.data(), sizeof(double) * len.size(), hipMemcpyHostToDevice,
                           b->stream));
    FinalizeArgs f{};
    f.acc = b->d_diag;
    f.nslots = b->nslots_diag;
    f.slot_stride = b->nrows * b->G;
    f.slot_len = b->d_slot_len;
    f.G = b->G;
    f.gs = b->P / b->G;
    f.M = b->nrows;
    f.comps = 1;
    f.out_index = b->d_orig;
    f.gstride = 1;
    f.mstride = b->G;
    f.est = want_max ? nullptr : b->d_est;   // a stop check needs only the per-row ratios
    f.se = want_max ? nullptr : b->d_se;
    f.val_group = b->d_row_mat;
    f.slot_len_stride = b->nslots_diag;
    f.rel_out = want_max ? b->d_rel : nullptr;
    BHIP(b, launch_finalize_groups(f, b->stream));
    if (want_max) {
        BHIP(b, launch_segment_max(b->d_rel, b->d_row0, b->M, b->d_mrel, b->stream));
        BHIP(b, hipMemcpyAsync(b->mrel.data(), b->d_mrel, sizeof(double) * b->M, hipMemcpyDeviceToHost, b->stream));
        BHIP(b, hipStreamSynchronize(b->stream));
    }
    return MCINV_OK;
}

mcinv_status check_batch(mcinv_batch* b)
{
    if (!b) return bfail(nullptr, MCINV_EINVAL, "null batch");
    BHIP(b, hipSetDevice(b->cfg.device));
    return commit(b);
}

}  // namespace

extern "C" {

mcinv_status mcinv_batch_create(const mcinv_batch_config* cfg, int64_t n_matrices, mcinv_batch** out)
try {
    if (!cfg || !out) return bfail(nullptr, MCINV_EINVAL, "null argument");
    *out = nullptr;
    const int32_t P = (int32_t)cfg->n_pairs;
    if (P != 16 && P != 32 && P != 64 && P != 128 && P != 256)
        return bfail(nullptr, MCINV_EINVAL, "batched form: n_pairs must be 16, 32, 64, 128 or 256");
    const int32_t G = cfg->n_groups;
    if (G < 1 || P % G != 0 || P / G < 4 || ((P / G) & (P / G - 1)) != 0)
        return bfail(nullptr, MCINV_EINVAL, "batched form: P/G must be a power of two >= 4");
    if (n_matrices < 1 || n_matrices > (1 << 20)) return bfail(nullptr, MCINV_EINVAL, "bad matrix count");
    if (cfg->noise < 0 || cfg->noise > 2) return bfail(nullptr, MCINV_EINVAL, "unknown noise kind");
    if (cfg->rows_per_item < 0 || cfg->grab < 0) return bfail(nullptr, MCINV_EINVAL, "bad schedule");
    if (cfg->schedule != MCINV_SCHEDULE_PHASED && cfg->schedule != MCINV_SCHEDULE_PERSISTENT)
        return bfail(nullptr, MCINV_EINVAL, "unknown schedule");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || cfg->device < 0 || cfg->device >= ndev)
        return bfail(nullptr, MCINV_EDEVICE, "no such HIP device");
    // the owner destroys a partly built context on every early return or exception
    std::unique_ptr<mcinv_batch, void (*)(mcinv_batch*)> owner(new mcinv_batch(), mcinv_batch_destroy);
    mcinv_batch* b = owner.get();
    b->cfg = *cfg;
    b->M = n_matrices;
    b->P = P;
    b->G = G;
    b->lane_shift = 0;
    while ((1 << b->lane_shift) < P / 4) ++b->lane_shift;
    b->prep.resize(n_matrices);
    b->loaded.assign(n_matrices, false);
    b->nslots_diag = G >= 16 ? 1 : kDiagSlotsSmallG;
    b->schedule = cfg->schedule;
    if (cfg->rows_per_item > 0) b->rows_per_item = cfg->rows_per_item;
    if (cfg->grab > 0) b->grab = cfg->grab;
    auto bail = [&](const char* msg) {
        g_berror = msg;
        return MCINV_EDEVICE;
    };
    if (hipSetDevice(cfg->device) != hipSuccess) return bail("hipSetDevice failed");
    if (cfg->stream) {
        b->stream = (hipStream_t)cfg->stream;
    } else {
        if (hipStreamCreate(&b->stream) != hipSuccess) return bail("hipStreamCreate failed");
        b->own_stream = true;
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, cfg->device) != hipSuccess) return bail("hipGetDeviceProperties failed");
    b->grid = prop.multiProcessorCount * batch_kernel_occupancy();
    if (hipMalloc((void**)&b->d_clock, sizeof(BatchClock)) != hipSuccess ||
        hipMalloc((void**)&b->d_flag, sizeof(int32_t)) != hipSuccess ||
        hipMalloc((void**)&b->d_slot_len, sizeof(double) * std::max(kBlockSlots, kDiagSlotsSmallG)) != hipSuccess)
        return bail("device allocation failed");
    if (hipMemsetAsync(b->d_clock, 0, sizeof(BatchClock), b->stream) != hipSuccess ||
        hipMemsetAsync(b->d_flag, 0, sizeof(int32_t), b->stream) != hipSuccess ||
        hipStreamSynchronize(b->stream) != hipSuccess)
        return bail("initial memset failed");
    *out = owner.release();
    return MCINV_OK;
} catch (...) {
    return mcinv::exception_status([&](mcinv_status s_, const std::string& m_) { bfail(nullptr, s_, m_); });
}

void mcinv_batch_destroy(mcinv_batch* b)
{
    if (!b) return;
    (void)hipSetDevice(b->cfg.device);
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    drop_graphs(b);
    bfree(b->d_rows);
    bfree(b->d_ent);
    bfree(b->d_sc);
    bfree(b->d_z);
    bfree(b->d_w);
    bfree(b->d_mats);
    bfree(b->d_mats_sample);
    bfree(b->d_done);
    bfree(b->d_clock);
    bfree(b->d_flag);
    bfree(b->d_orig);
    bfree(b->d_items_burn);
    bfree(b->d_items_sample);
    bfree(b->d_bI);
    bfree(b->d_bJ);
    bfree(b->d_diag);
    bfree(b->d_block);
    bfree(b->d_slot_len);
    bfree(b->d_est);
    bfree(b->d_se);
    bfree(b->d_row_mat);
    bfree(b->d_row0);
    bfree(b->d_rel);
    bfree(b->d_mrel);
    if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
}

mcinv_status mcinv_batch_load_csr(mcinv_batch* b, int64_t m, int64_t n, int64_t nnz, const int64_t* row_ptr,
                                  const int32_t* col_idx, const double* values)
try {
    if (!b) return bfail(nullptr, MCINV_EINVAL, "null batch");
    if (b->committed) return bfail(b, MCINV_ESTATE, "the batch is already committed (first sweep ran)");
    if (m < 0 || m >= b->M) return bfail(b, MCINV_EINVAL, "matrix index out of range");
    bool singular = false;
    const std::string why = prepare_matrix(n, nnz, row_ptr, col_idx, values, false, b->prep[m], &singular);
    if (!why.empty())
        return bfail(b, singular ? MCINV_ESINGULAR : MCINV_EINVAL, "matrix " + std::to_string(m) + ": " + why);
    b->loaded[m] = true;
    return MCINV_OK;
} catch (...) {
    return mcinv::exception_status([&](mcinv_status s_, const std::string& m_) { bfail(b, s_, m_); });
}

mcinv_status mcinv_batch_set_requested(mcinv_batch* b, uint32_t flags, int32_t block_dim, int64_t expected_samples)
try {
    BTRY(check_batch(b));
    if (flags & ~(MCINV_REQ_DIAG | MCINV_REQ_BLOCK))
        return bfail(b, MCINV_EINVAL, "the batched form estimates the diagonal and a block");
    if ((flags & MCINV_REQ_BLOCK) && (block_dim < 1 || block_dim > 128))
        return bfail(b, MCINV_EINVAL, "block_dim must be in [1, 128]");
    if (flags & MCINV_REQ_BLOCK)
        for (int64_t m = 0; m < b->M; ++m)
            if (b->prep[m].n < block_dim) return bfail(b, MCINV_EINVAL, "a matrix is smaller than block_dim");
    BHIP(b, hipStreamSynchronize(b->stream));
    bfree(b->d_diag);
    bfree(b->d_block);
    bfree(b->d_bI);
    bfree(b->d_bJ);
    b->flags = flags;
    b->bdim = (flags & MCINV_REQ_BLOCK) ? block_dim : 0;
    b->batch_len = std::max<int64_t>(1, (expected_samples + kBlockSlots - 1) / kBlockSlots);
    if (flags & MCINV_REQ_DIAG) {
        const size_t cnt = (size_t)b->nslots_diag * b->nrows * b->G;
        BTRY(balloc(b, &b->d_diag, cnt));
        BHIP(b, hipMemsetAsync(b->d_diag, 0, cnt * sizeof(double), b->stream));
    }
    if (b->bdim > 0) {
        // default block: the last block_dim rows and columns of each matrix
        b->hI.assign((size_t)b->M * b->bdim, 0);
        for (int64_t m = 0; m < b->M; ++m)
            for (int32_t r = 0; r < b->bdim; ++r)
                b->hI[m * b->bdim + r] = b->row0[m] + b->prep[m].pos[b->prep[m].n - b->bdim + r];
        b->hJ = b->hI;
        BTRY(bupload(b, &b->d_bI, b->hI));
        BTRY(bupload(b, &b->d_bJ, b->hJ));
        const size_t cnt = (size_t)kBlockSlots * b->M * b->bdim * b->bdim;
        BTRY(balloc(b, &b->d_block, cnt));
        BHIP(b, hipMemsetAsync(b->d_block, 0, cnt * sizeof(double), b->stream));
    }
    const int64_t cap = std::max<int64_t>(b->nrows, (int64_t)b->bdim * b->bdim);
    bfree(b->d_est);
    bfree(b->d_se);
    BTRY(balloc(b, &b->d_est, (size_t)cap));
    BTRY(balloc(b, &b->d_se, (size_t)cap));
    b->samples = 0;
    // every matrix takes part again, from zero samples
    std::fill(b->active.begin(), b->active.end(), (uint8_t)1);
    std::fill(b->msamples.begin(), b->msamples.end(), (int64_t)0);
    std::fill(b->mrel.begin(), b->mrel.end(), (double)INFINITY);
    // the device clock's sample count restarts with the accumulators
    BatchClock clk{};
    BHIP(b, hipMemcpyAsync(&clk, b->d_clock, sizeof(clk), hipMemcpyDeviceToHost, b->stream));
    BHIP(b, hipStreamSynchronize(b->stream));
    clk.sample = 0;
    BHIP(b, hipMemcpyAsync(b->d_clock, &clk, sizeof(clk), hipMemcpyHostToDevice, b->stream));
    BTRY(build_items(b));
    BHIP(b, hipStreamSynchronize(b->stream));
    b->requested = true;
    return MCINV_OK;
} catch (...) {
    return mcinv::exception_status([&](mcinv_status s_, const std::string& m_) { bfail(b, s_, m_); });
}

mcinv_status mcinv_batch_set_block(mcinv_batch* b, int64_t m, const int64_t* rows, const int64_t* cols)
try {
    BTRY(check_batch(b));
    if (!b->requested || b->bdim == 0) return bfail(b, MCINV_ESTATE, "request MCINV_REQ_BLOCK first");
    if (m < 0 || m >= b->M || !rows || !cols) return bfail(b, MCINV_EINVAL, "bad arguments");
    if (b->samples > 0) return bfail(b, MCINV_ESTATE, "set blocks before sampling");
    for (int32_t r = 0; r < b->bdim; ++r) {
        if (rows[r] < 0 || rows[r] >= b->prep[m].n || cols[r] < 0 || cols[r] >= b->prep[m].n)
            return bfail(b, MCINV_EINVAL, "block index out of range");
        b->hI[m * b->bdim + r] = b->row0[m] + b->prep[m].pos[rows[r]];
        b->hJ[m * b->bdim + r] = b->row0[m] + b->prep[m].pos[cols[r]];
    }
    BHIP(b, hipMemcpyAsync(b->d_bI + m * b->bdim, b->hI.data() + m * b->bdim, sizeof(int64_t) * b->bdim,
                           hipMemcpyHostToDevice, b->stream));
    BHIP(b, hipMemcpyAsync(b->d_bJ + m * b->bdim, b->hJ.data() + m * b->bdim, sizeof(int64_t) * b->bdim,
                           hipMemcpyHostToDevice, b->stream));
    BHIP(b, hipStreamSynchronize(b->stream));
    return MCINV_OK;
} catch (...) {
    return mcinv::exception_status([&](mcinv_status s_, const std::string& m_) { bfail(b, s_, m_); });
}

mcinv_status mcinv_batch_burn_in(mcinv_batch* b, int64_t sweeps)
try {
    BTRY(check_batch(b));
    if (sweeps < 0) return bfail(b, MCINV_EINVAL, "negative sweep count");
    hipEvent_t e0, e1;
    BHIP(b, hipEventCreate(&e0));
    BHIP(b, hipEventCreate(&e1));
    BHIP(b, hipEventRecord(e0, b->stream));
    BTRY(run_sweeps(b, sweeps, false));
    BHIP(b, hipEventRecord(e1, b->stream));
    BTRY(check_after(b));
    float ms = 0.f;
    BHIP(b, hipEventElapsedTime(&ms, e0, e1));
    b->last_ms = ms;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return MCINV_OK;
} catch (...) {
    return mcinv::exception_status([&](mcinv_status s_, const std::string& m_) { bfail(b, s_, m_); });
}

mcinv_status mcinv_batch_burn_in_coupled(mcinv_batch* b, double tol, int64_t max_sweeps, int64_t* sweeps_done,
                                         double* max_diff)
try {
    BTRY(check_batch(b));
    if (!(tol > 0.0) || max_sweeps < 0) return bfail(b, MCINV_EINVAL, "tol must be > 0 and max_sweeps >= 0");
    // Difference chains of every matrix (eq 12: noiseless Gauss-Seidel from
    // x*_i = i, 1-based original index), 16 lanes per row, phased launches.
    constexpr int32_t kLd = 16;
    const size_t cnt = (size_t)b->nrows * kLd;
    std::vector<float> init(cnt);
    std::vector<int32_t> row_m((size_t)b->nrows);
    for (int64_t m = 0; m < b->M; ++m)
        for (int64_t q = 0; q < b->prep[m].n; ++q) {
            const int64_t g = b->row0[m] + q;
            row_m[g] = (int32_t)m;
            for (int32_t l = 0; l < kLd; ++l) init[g * kLd + l] = (float)(b->prep[m].perm[q] + 1);
        }
    float *dz = nullptr, *dw = nullptr;
    int32_t *d_rowm = nullptr, *flag2 = nullptr;
    BatchClock* clock2 = nullptr;
    unsigned long long* dmax = nullptr;
    auto release = [&]() {
        bfree(dz);
        bfree(dw);
        bfree(d_rowm);
        bfree(flag2);
        bfree(clock2);
        bfree(dmax);
    };
    mcinv_status st = MCINV_OK;
    if ((st = balloc(b, &dz, cnt)) != MCINV_OK || (st = balloc(b, &dw, cnt)) != MCINV_OK ||
        (st = bupload(b, &d_rowm, row_m)) != MCINV_OK || (st = balloc(b, &flag2, 1)) != MCINV_OK ||
        (st = balloc(b, &clock2, 1)) != MCINV_OK || (st = balloc(b, &dmax, (size_t)(2 * b->M))) != MCINV_OK) {
        release();
        return st;
    }
    hipError_t e = hipMemcpyAsync(dz, init.data(), sizeof(float) * cnt, hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(dw, init.data(), sizeof(float) * cnt, hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipMemsetAsync(flag2, 0, sizeof(int32_t), b->stream);
    if (e == hipSuccess) e = hipMemsetAsync(clock2, 0, sizeof(BatchClock), b->stream);
    BatchArgs a = make_args(b, 1, false);
    a.z = dz;
    a.w = dw;
    a.P = kLd;
    a.lane_shift = 2;
    a.G = 1;
    a.noise = kNoiseNone;
    a.clock = clock2;
    a.flag = flag2;
    a.diag = nullptr;
    a.block = nullptr;
    const std::vector<int64_t>& off = b->phase_off[0];
    std::vector<unsigned long long> bits((size_t)(2 * b->M));
    int64_t N = max_sweeps;
    double worst = INFINITY;
    for (int64_t k = 1; k <= max_sweeps && e == hipSuccess; ++k) {
        for (size_t p = 0; p + 1 < off.size() && e == hipSuccess; ++p)
            e = launch_batch_phase(a, a.items + off[p], off[p + 1] - off[p], b->phase_block[0][p], b->stream);
        if (e == hipSuccess) e = launch_batch_tick(clock2, false, b->stream);
        if (e == hipSuccess) e = hipMemsetAsync(dmax, 0, sizeof(unsigned long long) * 2 * b->M, b->stream);
        if (e == hipSuccess) e = launch_batch_max_abs(dz, b->nrows, kLd, d_rowm, dmax, b->stream);
        if (e == hipSuccess) e = launch_batch_max_abs(dw, b->nrows, kLd, d_rowm, dmax + b->M, b->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(bits.data(), dmax, sizeof(unsigned long long) * bits.size(), hipMemcpyDeviceToHost,
                               b->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
        if (e != hipSuccess) break;
        worst = 0.0;
        for (unsigned long long u : bits) {
            double d;
            std::memcpy(&d, &u, sizeof(double));
            worst = std::max(worst, d);
        }
        if (!std::isfinite(worst)) {
            release();
            return bfail(b, MCINV_EDIVERGED, "coupled paths diverge (sp(T) or sp(S) >= 1 for some matrix)");
        }
        if (worst < tol) {
            N = k;
            break;
        }
    }
    release();
    if (e != hipSuccess) return bfail(b, MCINV_EDEVICE, std::string("coupled burn-in: ") + hipGetErrorString(e));
    BTRY(mcinv_batch_burn_in(b, N));
    if (sweeps_done) *sweeps_done = N;
    if (max_diff) *max_diff = worst;
    return MCINV_OK;
} catch (...) {
    return mcinv::exception_status([&](mcinv_status s_, const std::string& m_) { bfail(b, s_, m_); });
}

mcinv_status mcinv_batch_sample(mcinv_batch* b, int64_t sweeps)
try {
    BTRY(check_batch(b));
    if (!b->requested) return bfail(b, MCINV_ESTATE, "call mcinv_batch_set_requested before sampling");
    if (sweeps < 0) return bfail(b, MCINV_EINVAL, "negative sweep count");
    hipEvent_t e0, e1;
    BHIP(b, hipEventCreate(&e0));
    BHIP(b, hipEventCreate(&e1));
    BHIP(b, hipEventRecord(e0, b->stream));
    BTRY(run_sweeps(b, sweeps, true));
    BHIP(b, hipEventRecord(e1, b->stream));
    BTRY(check_after(b));
    float ms = 0.f;
    BHIP(b, hipEventElapsedTime(&ms, e0, e1));
    b->last_ms = ms;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return MCINV_OK;
} catch (...) {
    return mcinv::exception_status([&](mcinv_status s_, const std::string& m_) { bfail(b, s_, m_); });
}

mcinv_status mcinv_batch_sample_until(mcinv_batch* b, double rel_se, int64_t max_sweeps, int64_t check_every,
                                      int64_t* sweeps_done, double* achieved)
try {
    BTRY(check_batch(b));
    if (!b->requested || !(b->flags & MCINV_REQ_DIAG))
        return bfail(b, MCINV_ESTATE, "sample_until needs MCINV_REQ_DIAG requested");
    if (check_every < 1 || max_sweeps < 0) return bfail(b, MCINV_EINVAL, "bad sweep counts");
    BTRY(check_stop_batches(b));
    int64_t done = 0;
    double maxrel = INFINITY;
    while (done < max_sweeps) {
        const int64_t chunk = std::min(check_every, max_sweeps - done);
        BTRY(run_sweeps(b, chunk, true));
        done += chunk;
        BTRY(finalize_diag_all(b, true));
        BTRY(check_after(b));
        maxrel = *std::max_element(b->mrel.begin(), b->mrel.end());
        if (maxrel <= rel_se) break;
    }
    if (sweeps_done) *sweeps_done = done;
    if (achieved) *achieved = maxrel;
    return MCINV_OK;
} catch (...) {
    return mcinv::exception_status([&](mcinv_status s_, const std::string& m_) { bfail(b, s_, m_); });
}

mcinv_status mcinv_batch_sample_until_each(mcinv_batch* b, double rel_se, int64_t max_sweeps, int64_t check_every,
                                           int64_t* sweeps_done, double* achieved)
try {
    BTRY(check_batch(b));
    if (!b->requested || !(b->flags & MCINV_REQ_DIAG))
        return bfail(b, MCINV_ESTATE, "sample_until_each needs MCINV_REQ_DIAG requested");
    if (check_every < 1 || max_sweeps < 0) return bfail(b, MCINV_EINVAL, "bad sweep counts");
    BTRY(check_stop_batches(b));
    int64_t done = 0;
    int64_t left = std::count(b->active.begin(), b->active.end(), (uint8_t)1);
    // Once a matrix has stopped, the item lists change at every few checks:
    // the chunks are then launched directly rather than captured and
    // instantiated as graphs for a single replay.
    bool graphs = true;
    while (done < max_sweeps && left > 0) {
        const int64_t chunk = std::min(check_every, max_sweeps - done);
        BTRY(run_sweeps(b, chunk, true, graphs));
        done += chunk;
        BTRY(finalize_diag_all(b, true));
        BTRY(check_after(b));
        bool stopped = false;
        for (int64_t m = 0; m < b->M; ++m)
            if (b->active[m] && b->mrel[m] <= rel_se) {
                b->active[m] = 0;
                stopped = true;
                --left;
            }
        // the remaining matrices' item lists (and the graphs replaying them)
        if (stopped) {
            BTRY(build_items(b));
            graphs = false;
        }
    }
    if (sweeps_done) *sweeps_done = done;
    if (achieved) *achieved = *std::max_element(b->mrel.begin(), b->mrel.end());
    return MCINV_OK;
} catch (...) {
    return mcinv::exception_status([&](mcinv_status s_, const std::string& m_) { bfail(b, s_, m_); });
}

mcinv_status mcinv_batch_matrix_samples(mcinv_batch* b, int64_t* samples, uint8_t* active)
try {
    BTRY(check_batch(b));
    if (samples) std::copy(b->msamples.begin(), b->msamples.end(), samples);
    if (active) std::copy(b->active.begin(), b->active.end(), active);
    return MCINV_OK;
} catch (...) {
    return mcinv::exception_status([&](mcinv_status s_, const std::string& m_) { bfail(b, s_, m_); });
}

mcinv_status mcinv_batch_read_estimates(mcinv_batch* b, int64_t m, uint32_t quantity, double* est, double* stderr_,
                                        int64_t capacity)
try {
    BTRY(check_batch(b));
    if (m < 0 || m >= b->M) return bfail(b, MCINV_EINVAL, "matrix index out of range");
    if (!b->requested || !(b->flags & quantity)) return bfail(b, MCINV_ESTATE, "quantity was not requested");
    int64_t count = 0, offset = 0;
    if (quantity == MCINV_REQ_DIAG) {
        count = b->prep[m].n;
        offset = b->row0[m];
        if (capacity < count) return bfail(b, MCINV_EINVAL, "capacity too small");
        BTRY(finalize_diag_all(b, false));
    } else if (quantity == MCINV_REQ_BLOCK) {
        count = (int64_t)b->bdim * b->bdim;
        if (capacity < count) return bfail(b, MCINV_EINVAL, "capacity too small");
        const std::vector<double> len = slot_lengths(b->msamples[m], b->batch_len, kBlockSlots);
        BHIP(b, hipMemcpyAsync(b->d_slot_len, len.data(), sizeof(double) * len.size(), hipMemcpyHostToDevice,
                               b->stream));
        FinalizeArgs f{};
        f.acc = b->d_block + m * count;
        f.nslots = kBlockSlots;
        f.slot_stride = b->M * count;
        f.slot_len = b->d_slot_len;
        f.G = 1;
        f.gs = b->P;
        f.M = count;
        f.comps = 1;
        f.est = b->d_est;
        f.se = b->d_se;
        BHIP(b, launch_finalize_flat(f, b->stream));
    } else {
        return bfail(b, MCINV_EINVAL, "quantity must be MCINV_REQ_DIAG or MCINV_REQ_BLOCK");
    }
    if (est) BHIP(b, hipMemcpyAsync(est, b->d_est + offset, sizeof(double) * count, hipMemcpyDeviceToHost, b->stream));
    if (stderr_)
        BHIP(b, hipMemcpyAsync(stderr_, b->d_se + offset, sizeof(double) * count, hipMemcpyDeviceToHost, b->stream));
    BHIP(b, hipStreamSynchronize(b->stream));
    return MCINV_OK;
} catch (...) {
    return mcinv::exception_status([&](mcinv_status s_, const std::string& m_) { bfail(b, s_, m_); });
}

mcinv_status mcinv_batch_read_labels(mcinv_batch* b, int64_t m, double* y, double* y_se, int64_t capacity)
try {
    BTRY(check_batch(b));
    if (m < 0 || m >= b->M) return bfail(b, MCINV_EINVAL, "matrix index out of range");
    const Prepared& pm = b->prep[m];
    const int64_t n = pm.n;
    if (capacity < n || !y || !y_se) return bfail(b, MCINV_EINVAL, "null output or capacity too small");
    std::vector<double> est((size_t)n), se((size_t)n);
    BTRY(mcinv_batch_read_estimates(b, m, MCINV_REQ_DIAG, est.data(), se.data(), n));
    // estimates are in original row order; c_ii is kept per sweep position
    for (int64_t i = 0; i < n; ++i) {
        const double d = pm.diag[(size_t)pm.pos[i]].real();
        y[i] = d * est[(size_t)i];
        y_se[i] = std::fabs(d) * se[(size_t)i];
    }
    return MCINV_OK;
} catch (...) {
    return mcinv::exception_status([&](mcinv_status s_, const std::string& m_) { bfail(b, s_, m_); });
}

mcinv_status mcinv_batch_read_state(mcinv_batch* b, int64_t m, int32_t which, float* host, int64_t bytes)
try {
    BTRY(check_batch(b));
    if (m < 0 || m >= b->M || (which != 0 && which != 1) || !host) return bfail(b, MCINV_EINVAL, "bad arguments");
    const int64_t n = b->prep[m].n;
    if (bytes < n * b->P * (int64_t)sizeof(float)) return bfail(b, MCINV_EINVAL, "host buffer too small");
    std::vector<float> tmp((size_t)n * b->P);
    BHIP(b, hipMemcpyAsync(tmp.data(), (which ? b->d_w : b->d_z) + b->row0[m] * b->P, tmp.size() * sizeof(float),
                           hipMemcpyDeviceToHost, b->stream));
    BHIP(b, hipStreamSynchronize(b->stream));
    for (int64_t i = 0; i < n; ++i)
        std::memcpy(host + i * b->P, tmp.data() + b->prep[m].pos[i] * b->P, sizeof(float) * b->P);
    return MCINV_OK;
} catch (...) {
    return mcinv::exception_status([&](mcinv_status s_, const std::string& m_) { bfail(b, s_, m_); });
}

mcinv_status mcinv_batch_autotune(mcinv_batch* b, int32_t sweeps_per_trial, int32_t* schedule,
                                  int32_t* rows_per_item, int32_t* grab, double* ms_per_sweep)
try {
    BTRY(check_batch(b));
    if (sweeps_per_trial < 1) return bfail(b, MCINV_EINVAL, "sweeps_per_trial must be >= 1");
    const int32_t rows_c[] = {16, 32, 64, 128, 256, 512, 1024};
    const int32_t grab_c[] = {1, 4};
    double best = INFINITY;
    int32_t best_r = b->rows_per_item, best_g = b->grab, best_s = b->schedule;
    hipEvent_t e0, e1;
    BHIP(b, hipEventCreate(&e0));
    BHIP(b, hipEventCreate(&e1));
    for (int32_t sched : {MCINV_SCHEDULE_PHASED, MCINV_SCHEDULE_PERSISTENT}) {
    bool first = true, skip = false;
    for (int32_t r : rows_c)
        for (int32_t g : grab_c) {
            if (sched == MCINV_SCHEDULE_PHASED && g != grab_c[0]) continue;  // grab is persistent-only
            if (skip) continue;
            b->schedule = sched;
            b->rows_per_item = r;
            b->grab = g;
            BTRY(build_items(b));
            BTRY(run_sweeps(b, 1, false, false));  // warm-up
            BHIP(b, hipEventRecord(e0, b->stream));
            BTRY(run_sweeps(b, sweeps_per_trial, false, false));
            BHIP(b, hipEventRecord(e1, b->stream));
            BTRY(check_after(b));
            float ms = 0.f;
            BHIP(b, hipEventElapsedTime(&ms, e0, e1));
            const double per = ms / sweeps_per_trial;
            // a schedule whose first candidate is over twice the best so far is not explored further
            if (first && per > 2.0 * best) skip = true;
            first = false;
            if (per < best) {
                best = per;
                best_r = r;
                best_g = g;
                best_s = sched;
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    b->rows_per_item = best_r;
    b->grab = best_g;
    b->schedule = best_s;
    BTRY(build_items(b));
    if (schedule) *schedule = best_s;
    if (rows_per_item) *rows_per_item = best_r;
    if (grab) *grab = best_g;
    if (ms_per_sweep) *ms_per_sweep = best;
    return MCINV_OK;
} catch (...) {
    return mcinv::exception_status([&](mcinv_status s_, const std::string& m_) { bfail(b, s_, m_); });
}

mcinv_status mcinv_batch_get_info(mcinv_batch* b, mcinv_batch_info* out)
try {
    if (!b || !out) return bfail(b, MCINV_EINVAL, "null argument");
    std::memset(out, 0, sizeof(*out));
    out->n_matrices = b->M;
    out->n_rows = b->nrows;
    out->nnz = b->nnz_total;
    out->n_pairs = b->P;
    out->n_groups = b->G;
    out->max_colors = b->max_colors;
    out->rows_per_item = b->rows_per_item;
    out->grab = b->grab;
    out->grid = b->grid;
    out->schedule = b->schedule;
    out->items_per_sweep = b->ips_sample > 0 ? b->ips_sample : b->ips_burn;
    out->sweeps_done = b->sweeps;
    out->samples_done = b->samples;
    out->last_call_ms = b->last_ms;
    return MCINV_OK;
} catch (...) {
    return mcinv::exception_status([&](mcinv_status s_, const std::string& m_) { bfail(b, s_, m_); });
}

const char* mcinv_batch_last_error(const mcinv_batch* b)
{
    return b ? b->err.c_str() : g_berror.c_str();
}

}  // extern "C"
