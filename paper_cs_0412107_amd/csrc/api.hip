// Host runtime and C-ABI of the mcinv library (declared in include/mcinv.h).
//
// load_csr prepares everything the sweep kernels read:
//   - validation (sorted columns, nonzero diagonal: Sec. 2.2 needs D regular),
//   - the transpose of C (eq 5 walks column i of C),
//   - one merged off-diagonal pattern per row (the union of row i and column i)
//     holding both coefficients u = c_ij/c_ii (eq 4) and
//     v = conj(c_ji)/conj(c_ii) (eq 5), so a neighbour is visited once,
//   - a greedy first-fit colouring of that pattern in natural row order and the
//     position order (colour, row): a symmetric permutation of C,
//   - noise scales a, b with a conj(b) = 1/c_ii, computed in fp64 and rounded
//     to the sweep precision.
// burn_in / sample enqueue one kernel per colour per sweep on the context's
// stream; moments are fused into the sweep (diagonal, trace) or follow it
// (block, entries, per-sweep trace reduction).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "../../include/mcinv.h"
#include "boundary.h"
#include "device_common.h"
#include "prep.h"
#include "coupling.h"
#include "moments.h"
#include "sweep.h"

using namespace mcinv;

namespace {

thread_local std::string g_error;

constexpr int64_t kSlotsSmallG = 64;     // time batches when there are < 16 groups
constexpr int64_t kSmallLaunchRows = 4096;  // a colour launch below this many row-waves is "small"
constexpr double kGuardThreshold = 1e30;
constexpr int kLaunchOrders = 4;       // workgroup orders mcinv_tune_launch compares

}  // namespace

namespace mcinv {
void set_context_free_error(const std::string& msg) { g_error = msg; }
}  // namespace mcinv

struct mcinv_ctx {
    mcinv_config cfg{};
    hipStream_t stream = nullptr;
    bool own_stream = false;
    hipStream_t side = nullptr;   // the coupled burn-in's difference iteration (created on first use)
    bool cplx = false;
    size_t elem = 0;
    int comps = 1;

    int64_t P = 0, ld = 0, G = 1, gs = 1, lg_shift = 6, A = 1, cpt = 1, ntiles = 1, pairs_per_col = 256;
    int64_t pass_tiles = 1;   // pair tiles per pass (all colours of a pass before the next)

    // matrix
    bool loaded = false;
    bool real_values = true;
    int64_t n = 0, nnz = 0, n_off = 0;
    int32_t ncolors = 0;
    uint64_t value_hash = 0;     // FNV-1a of the prepared coefficients (checkpoint fingerprint)
    uint64_t q_hash = 0;         // FNV-1a of Q's position-order pattern and values
    std::vector<int64_t> perm, pos, color_ptr, tpart_off;
    std::vector<int32_t> color;
    int64_t npart = 0;

    // device: matrix and state
    RowRec* d_rows = nullptr;
    void* d_ent = nullptr;
    void* d_sc = nullptr;
    void* d_z = nullptr;
    void* d_w = nullptr;
    int64_t* d_perm = nullptr;
    int32_t* d_flag = nullptr;

    // requests
    uint32_t flags = 0;
    bool requested = false;
    int64_t nI = 0, nJ = 0, ne = 0;
    int64_t* d_I = nullptr;
    int64_t* d_J = nullptr;
    int64_t* d_ei = nullptr;
    int64_t* d_ej = nullptr;

    // accumulators
    int64_t nslots = 1, batch_len = 1, samples = 0, sweeps = 0;
    std::vector<double> slot_len;
    double* d_slot_len = nullptr;
    double* d_diag = nullptr;
    double* d_block = nullptr;
    double* d_entries = nullptr;
    double* d_tpart = nullptr;
    double* d_partial = nullptr;
    uint32_t* d_counter = nullptr;
    double* d_series = nullptr;
    int64_t series_cap = 0;
    double* d_est = nullptr;
    double* d_se = nullptr;
    int64_t est_cap = 0;
    unsigned long long* d_maxrel = nullptr;
    double* d_geyer = nullptr;
    uint8_t* d_stop = nullptr;   // rows the stop check covers (null: every row)
    // general trace matrix Q (eq tr), position order
    int64_t* d_qrp = nullptr;
    int64_t* d_qcol = nullptr;
    void* d_qval = nullptr;
    int64_t q_nnz = -1;          // -1: no Q loaded
    double* d_qpart = nullptr;
    double* d_qseries = nullptr;
    int64_t qseries_cap = 0;

    // profiling
    std::vector<hipEvent_t> events;
    double sweep_ms = 0.0, moment_ms = 0.0;
    int64_t sweep_launches = 0, moment_launches = 0;

    std::string err;

    int64_t diag_slot_stride() const { return ntiles * n * cpt * comps; }
    int64_t block_slot_stride() const { return G * nI * nJ * comps; }
    int64_t entry_slot_stride() const { return G * ne * comps; }
};

namespace {

// FNV-1a over raw bytes (checkpoint fingerprints).
uint64_t fnv1a(uint64_t h, const void* p, size_t bytes)
{
    const unsigned char* b = (const unsigned char*)p;
    for (size_t k = 0; k < bytes; ++k) {
        h ^= b[k];
        h *= 1099511628211ull;
    }
    return h;
}
constexpr uint64_t kFnvBasis = 1469598103934665603ull;

mcinv_status fail(mcinv_ctx* c, mcinv_status code, const std::string& msg)
{
    if (c)
        c->err = msg;
    else
        g_error = msg;
    return code;
}

#define HIP_TRY(c, expr)                                                                        \
    do {                                                                                        \
        hipError_t e_ = (expr);                                                                 \
        if (e_ != hipSuccess)                                                                   \
            return fail((c), e_ == hipErrorOutOfMemory ? MCINV_ENOMEM : MCINV_EDEVICE,          \
                        std::string(#expr) + ": " + hipGetErrorString(e_));                     \
    } while (0)

#define MC_TRY(expr)                    \
    do {                                \
        mcinv_status s_ = (expr);       \
        if (s_ != MCINV_OK) return s_;  \
    } while (0)

template <typename T>
void dfree(T*& p)
{
    if (p) (void)hipFree((void*)p);
    p = nullptr;
}

void free_requests(mcinv_ctx* c)
{
    dfree(c->d_I);
    dfree(c->d_J);
    dfree(c->d_ei);
    dfree(c->d_ej);
    dfree(c->d_diag);
    dfree(c->d_block);
    dfree(c->d_entries);
    dfree(c->d_tpart);
    dfree(c->d_series);
    dfree(c->d_slot_len);
    dfree(c->d_qpart);
    dfree(c->d_qseries);
    c->qseries_cap = 0;
    c->series_cap = 0;
    c->requested = false;
    c->flags = 0;
    c->nI = c->nJ = c->ne = 0;
}

void free_matrix(mcinv_ctx* c)
{
    free_requests(c);
    dfree(c->d_rows);
    dfree(c->d_ent);
    dfree(c->d_sc);
    dfree(c->d_z);
    dfree(c->d_w);
    dfree(c->d_perm);
    dfree(c->d_stop);
    dfree(c->d_qrp);
    dfree(c->d_qcol);
    dfree(c->d_qval);
    c->q_nnz = -1;
    dfree(c->d_est);
    dfree(c->d_se);
    c->est_cap = 0;
    c->loaded = false;
}

mcinv_status set_device(mcinv_ctx* c)
{
    HIP_TRY(c, hipSetDevice(c->cfg.device));
    return MCINV_OK;
}

template <typename T>
mcinv_status dalloc(mcinv_ctx* c, T** p, size_t count)
{
    *p = nullptr;
    if (count == 0) count = 1;
    HIP_TRY(c, hipMalloc((void**)p, count * sizeof(T)));
    return MCINV_OK;
}

template <typename T>
mcinv_status upload(mcinv_ctx* c, T** p, const std::vector<T>& h)
{
    MC_TRY(dalloc(c, p, h.size()));
    if (!h.empty()) HIP_TRY(c, hipMemcpyAsync(*p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, c->stream));
    return MCINV_OK;
}

template <typename V>
mcinv_status upload_matrix(mcinv_ctx* c, const Prepared& h)
{
    std::vector<Entry<V>> ent(h.ent.size());
    for (size_t e = 0; e < ent.size(); ++e) {
        ent[e].col = (int32_t)h.ent[e].col;
        ent[e].pad = 0;
        ent[e].u = cast_val<V>(h.ent[e].u);
        ent[e].v = cast_val<V>(h.ent[e].v);
    }
    std::vector<Scales<V>> sc(h.a.size());
    for (size_t q = 0; q < sc.size(); ++q) {
        sc[q].a = cast_val<V>(h.a[q]);
        sc[q].b = cast_val<V>(h.b[q]);
    }
    Entry<V>* d_ent = nullptr;
    Scales<V>* d_sc = nullptr;
    MC_TRY(upload(c, &c->d_rows, h.rows));
    MC_TRY(upload(c, &d_ent, ent));
    c->d_ent = d_ent;
    MC_TRY(upload(c, &d_sc, sc));
    c->d_sc = d_sc;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return MCINV_OK;
}

// ------------------------------------------------------------ the sweeps --
int64_t qtrace_partials(const mcinv_ctx* c)
{
    const int64_t rows_per_block = 4 * kQRowsPerWave;
    return (c->n + rows_per_block - 1) / rows_per_block * c->ntiles;
}

mcinv_status grow_series(mcinv_ctx* c, int64_t need, double** series, int64_t* series_cap)
{
    if (need <= *series_cap) return MCINV_OK;
    int64_t cap = std::max<int64_t>(4096, *series_cap);
    while (cap < need) cap *= 2;
    double* nb = nullptr;
    MC_TRY(dalloc(c, &nb, (size_t)(cap * c->comps)));
    if (*series && c->samples > 0)
        HIP_TRY(c, hipMemcpyAsync(nb, *series, sizeof(double) * c->samples * c->comps, hipMemcpyDeviceToDevice,
                                  c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    dfree(*series);
    *series = nb;
    *series_cap = cap;
    return MCINV_OK;
}

mcinv_status grow_series(mcinv_ctx* c, int64_t need) { return grow_series(c, need, &c->d_series, &c->series_cap); }

hipEvent_t take_event(mcinv_ctx* c, size_t& next)
{
    if (next >= c->events.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        c->events.push_back(e);
    }
    return c->events[next++];
}

// Merge the time-batch clusters pairwise when all slots are full.
mcinv_status advance_slot(mcinv_ctx* c, int64_t* slot)
{
    int64_t b = c->samples / c->batch_len;
    if (c->nslots > 1 && b >= c->nslots) {
        const int64_t half = c->nslots / 2;
        if (c->d_diag) HIP_TRY(c, launch_merge_slots(c->d_diag, c->diag_slot_stride(), half, c->stream));
        if (c->d_block) HIP_TRY(c, launch_merge_slots(c->d_block, c->block_slot_stride(), half, c->stream));
        if (c->d_entries) HIP_TRY(c, launch_merge_slots(c->d_entries, c->entry_slot_stride(), half, c->stream));
        for (int64_t m = 0; m < half; ++m) c->slot_len[m] = c->slot_len[2 * m] + c->slot_len[2 * m + 1];
        for (int64_t m = half; m < c->nslots; ++m) c->slot_len[m] = 0.0;
        c->batch_len *= 2;
        b = c->samples / c->batch_len;
    }
    if (c->nslots == 1) b = 0;
    *slot = b;
    return MCINV_OK;
}

template <typename V>
mcinv_status run_sweeps(mcinv_ctx* c, int64_t nsw, bool sample, V* z, V* w, int64_t ld, int64_t P,
                        int32_t noise, int32_t* flag, bool use_counters)
{
    SweepArgs<V> a{};
    a.rows = c->d_rows;
    a.ent = (const Entry<V>*)c->d_ent;
    a.sc = (const Scales<V>*)c->d_sc;
    a.z = z;
    a.w = w;
    a.ld = ld;
    a.P = P;
    a.key0 = (uint32_t)(c->cfg.seed & 0xffffffffu);
    a.key1 = (uint32_t)(c->cfg.seed >> 32);
    a.stream = c->cfg.stream_id;
    a.pair_block0 = (uint32_t)(c->cfg.pair_offset >> 2);
    a.noise = noise;
    a.lg_shift = (int32_t)c->lg_shift;
    a.n = c->n;
    a.flag = flag;
    a.thresh = (typename Real<V>::type)kGuardThreshold;
    a.xcd_order = c->cfg.xcd_order;

    const bool prof = c->cfg.profile != 0 && use_counters;
    int64_t launches_per_sweep = 0;   // sweep-kernel launches between one timed sweep's events
    size_t next_ev = 0;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> sweep_ev, mom_ev;

    for (int64_t s = 0; s < nsw; ++s) {
        const int64_t k = use_counters ? c->sweeps + s : s;
        int64_t slot = 0;
        if (sample) MC_TRY(advance_slot(c, &slot));
        a.sweep = (uint32_t)k;
        const bool want_diag = sample && (c->flags & MCINV_REQ_DIAG);
        const bool want_trace = sample && (c->flags & MCINV_REQ_TRACE);
        a.diag = want_diag ? c->d_diag + slot * c->diag_slot_stride() : nullptr;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (prof) {
            e0 = take_event(c, next_ev);
            e1 = take_event(c, next_ev);
            if (e0) HIP_TRY(c, hipEventRecord(e0, c->stream));
        }
        // Passes over groups of pair tiles: within a pass every colour runs for
        // the pass's tiles, so their state slices stay cache-resident across
        // colours.  Trailing small colours (too few rows to fill a launch for
        // one pass) run once over all tiles after the passes; per tile the
        // colour order is unchanged.
        const int64_t T = (ld + kPairsPerWave - 1) / kPairsPerWave;
        const int64_t pt = use_counters ? std::min<int64_t>(std::max<int64_t>(c->pass_tiles, 1), T) : T;
        int32_t cs = c->ncolors;
        while (cs > 0 && (c->color_ptr[cs] - c->color_ptr[cs - 1]) * pt < kSmallLaunchRows) --cs;
        if (pt >= T) cs = c->ncolors;
        launches_per_sweep = (T + pt - 1) / pt * cs + (c->ncolors - cs);
        a.nt_stores = c->cfg.stores == 1 || (c->cfg.stores == 0 && pt >= T);
        for (int64_t t0 = 0; t0 < T; t0 += pt) {
            for (int32_t col = 0; col < cs; ++col) {
                a.row_begin = c->color_ptr[col];
                a.row_end = c->color_ptr[col + 1];
                a.tile0 = t0;
                a.tpart = want_trace ? c->d_tpart + c->tpart_off[col] * c->comps : nullptr;
                HIP_TRY(c, launch_sweep<V>(a, std::min(pt, T - t0), sample, c->cfg.hermitian != 0, c->stream));
            }
        }
        for (int32_t col = cs; col < c->ncolors; ++col) {
            a.row_begin = c->color_ptr[col];
            a.row_end = c->color_ptr[col + 1];
            a.tile0 = 0;
            a.tpart = want_trace ? c->d_tpart + c->tpart_off[col] * c->comps : nullptr;
            HIP_TRY(c, launch_sweep<V>(a, T, sample, c->cfg.hermitian != 0, c->stream));
        }
        if (prof && e1) {
            HIP_TRY(c, hipEventRecord(e1, c->stream));
            sweep_ev.emplace_back(e0, e1);
        }
        if (!sample) continue;

        if (want_trace) {
            MC_TRY(grow_series(c, c->samples + 1));
            HIP_TRY(c, launch_reduce_sum(c->d_tpart, c->npart, c->comps, c->d_partial, c->d_counter,
                                         c->d_series + c->samples * c->comps, c->stream));
        }
        if (c->flags & MCINV_REQ_QTRACE) {
            MC_TRY(grow_series(c, c->samples + 1, &c->d_qseries, &c->qseries_cap));
            QTraceArgs<V> qa{};
            qa.z = z;
            qa.w = w;
            qa.ld = ld;
            qa.P = P;
            qa.n = c->n;
            qa.qrp = c->d_qrp;
            qa.qcol = c->d_qcol;
            qa.qval = (const V*)c->d_qval;
            qa.part = c->d_qpart;
            HIP_TRY(c, launch_qtrace<V>(qa, c->stream));
            HIP_TRY(c, launch_reduce_sum(c->d_qpart, qtrace_partials(c), c->comps, c->d_partial, c->d_counter,
                                         c->d_qseries + c->samples * c->comps, c->stream));
        }
        hipEvent_t m0 = nullptr, m1 = nullptr;
        const bool any_moment = (c->flags & MCINV_REQ_BLOCK) || (c->flags & MCINV_REQ_ENTRIES);
        if (prof && any_moment) {
            m0 = take_event(c, next_ev);
            m1 = take_event(c, next_ev);
            if (m0) HIP_TRY(c, hipEventRecord(m0, c->stream));
        }
        if ((c->flags & MCINV_REQ_BLOCK) && c->nI > 0 && c->nJ > 0) {
            BlockArgs<V> ba{};
            ba.z = z;
            ba.w = w;
            ba.ld = ld;
            ba.I = c->d_I;
            ba.J = c->d_J;
            ba.nI = c->nI;
            ba.nJ = c->nJ;
            ba.gs = c->gs;
            ba.G = c->G;
            ba.acc = c->d_block + slot * c->block_slot_stride();
            if constexpr (std::is_same<V, float>::value) {
                if (c->cfg.moments == MCINV_MOMENTS_BF16X3)
                    HIP_TRY(c, launch_block_bf16x3(ba, c->stream));
                else
                    HIP_TRY(c, launch_block_fp64<V>(ba, c->stream));
            } else {
                HIP_TRY(c, launch_block_fp64<V>(ba, c->stream));
            }
        }
        if ((c->flags & MCINV_REQ_ENTRIES) && c->ne > 0)
            HIP_TRY(c, launch_entries<V>(z, w, ld, c->d_ei, c->d_ej, c->ne, c->gs, c->G,
                                         c->d_entries + slot * c->entry_slot_stride(), c->stream));
        if (prof && m1) {
            HIP_TRY(c, hipEventRecord(m1, c->stream));
            mom_ev.emplace_back(m0, m1);
        }
        c->slot_len[slot] += 1.0;
        c->samples += 1;
    }
    if (prof) {
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        for (auto& pr : sweep_ev) {
            float ms = 0.f;
            HIP_TRY(c, hipEventElapsedTime(&ms, pr.first, pr.second));
            c->sweep_ms += ms;
            c->sweep_launches += launches_per_sweep;
        }
        for (auto& pr : mom_ev) {
            float ms = 0.f;
            HIP_TRY(c, hipEventElapsedTime(&ms, pr.first, pr.second));
            c->moment_ms += ms;
            c->moment_launches += 1;
        }
    }
    return MCINV_OK;
}

// The w state: z itself in hermitian mode (w = z at every step).
void* w_state(mcinv_ctx* c) { return c->cfg.hermitian ? c->d_z : c->d_w; }

mcinv_status dispatch_sweeps(mcinv_ctx* c, int64_t nsw, bool sample)
{
    void* const wst = w_state(c);
    switch (c->cfg.sweep_dtype) {
    case MCINV_R32:
        return run_sweeps<float>(c, nsw, sample, (float*)c->d_z, (float*)wst, c->ld, c->P, c->cfg.noise,
                                 c->d_flag, true);
    case MCINV_R64:
        return run_sweeps<double>(c, nsw, sample, (double*)c->d_z, (double*)wst, c->ld, c->P, c->cfg.noise,
                                  c->d_flag, true);
    case MCINV_C64:
        return run_sweeps<Cx<float>>(c, nsw, sample, (Cx<float>*)c->d_z, (Cx<float>*)wst, c->ld, c->P,
                                     c->cfg.noise, c->d_flag, true);
    default:
        return run_sweeps<Cx<double>>(c, nsw, sample, (Cx<double>*)c->d_z, (Cx<double>*)wst, c->ld, c->P,
                                      c->cfg.noise, c->d_flag, true);
    }
}

mcinv_status check_flag(mcinv_ctx* c)
{
    int32_t flag = 0;
    HIP_TRY(c, hipMemcpyAsync(&flag, c->d_flag, sizeof(flag), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (flag) return fail(c, MCINV_EDIVERGED, "chain state became non-finite or exceeded 1e30 (sp(T) or sp(S) >= 1?)");
    return MCINV_OK;
}

mcinv_status ensure_est(mcinv_ctx* c, int64_t values)
{
    if (values <= c->est_cap) return MCINV_OK;
    dfree(c->d_est);
    dfree(c->d_se);
    MC_TRY(dalloc(c, &c->d_est, (size_t)(values * 2)));
    MC_TRY(dalloc(c, &c->d_se, (size_t)values));
    c->est_cap = values;
    return MCINV_OK;
}

mcinv_status finalize_diag(mcinv_ctx* c, bool want_max)
{
    MC_TRY(ensure_est(c, c->n));
    HIP_TRY(c, hipMemcpyAsync(c->d_slot_len, c->slot_len.data(), sizeof(double) * c->nslots,
                              hipMemcpyHostToDevice, c->stream));
    if (want_max) HIP_TRY(c, hipMemsetAsync(c->d_maxrel, 0, sizeof(unsigned long long), c->stream));
    FinalizeArgs f{};
    f.acc = c->d_diag;
    f.nslots = c->nslots;
    f.slot_stride = c->diag_slot_stride();
    f.slot_len = c->d_slot_len;
    f.G = c->G;
    f.gs = c->gs;
    f.M = c->n;
    f.A = c->A;
    f.cpt = c->cpt;
    f.pairs_per_col = c->pairs_per_col;
    f.comps = c->comps;
    f.out_index = c->d_perm;
    f.est = c->d_est;
    f.se = c->d_se;
    f.max_rel = want_max ? c->d_maxrel : nullptr;
    f.stop_mask = c->d_stop;
    HIP_TRY(c, launch_finalize_diag(f, c->stream));
    return MCINV_OK;
}

mcinv_status finalize_flat(mcinv_ctx* c, const double* acc, int64_t M, int64_t stride)
{
    MC_TRY(ensure_est(c, M));
    HIP_TRY(c, hipMemcpyAsync(c->d_slot_len, c->slot_len.data(), sizeof(double) * c->nslots,
                              hipMemcpyHostToDevice, c->stream));
    FinalizeArgs f{};
    f.acc = acc;
    f.nslots = c->nslots;
    f.slot_stride = stride;
    f.slot_len = c->d_slot_len;
    f.G = c->G;
    f.gs = c->gs;
    f.M = M;
    f.comps = c->comps;
    f.est = c->d_est;
    f.se = c->d_se;
    HIP_TRY(c, launch_finalize_flat(f, c->stream));
    return MCINV_OK;
}

size_t elem_size(int32_t dt)
{
    switch (dt) {
    case MCINV_R32: return 4;
    case MCINV_R64: return 8;
    case MCINV_C64: return 8;
    case MCINV_C128: return 16;
    default: return 0;
    }
}

mcinv_status check_ready(mcinv_ctx* c)
{
    if (!c) return fail(nullptr, MCINV_EINVAL, "null context");
    if (!c->loaded) return fail(c, MCINV_ESTATE, "no matrix loaded (call mcinv_load_csr first)");
    return set_device(c);
}

}  // namespace

// =========================================================================
extern "C" {

mcinv_status mcinv_create(const mcinv_config* cfg, mcinv_ctx** out)
try {
    if (!cfg || !out) return fail(nullptr, MCINV_EINVAL, "null argument");
    *out = nullptr;
    if (elem_size(cfg->sweep_dtype) == 0) return fail(nullptr, MCINV_EINVAL, "unknown sweep dtype");
    if (cfg->noise < 0 || cfg->noise > 2) return fail(nullptr, MCINV_EINVAL, "unknown noise kind");
    if (cfg->moments != MCINV_MOMENTS_FP64 && cfg->moments != MCINV_MOMENTS_BF16X3)
        return fail(nullptr, MCINV_EINVAL, "unknown moments mode");
    if (cfg->moments == MCINV_MOMENTS_BF16X3 && cfg->sweep_dtype != MCINV_R32)
        return fail(nullptr, MCINV_EINVAL, "bf16x3 block moments need a real fp32 sweep");
    if (cfg->n_pairs < 1 || cfg->n_pairs > (int64_t)1 << 30) return fail(nullptr, MCINV_EINVAL, "n_pairs out of range");
    if (cfg->xcd_order < 0 || cfg->xcd_order > 3) return fail(nullptr, MCINV_EINVAL, "xcd_order must be 0 .. 3");
    if (cfg->stores < 0 || cfg->stores > 2) return fail(nullptr, MCINV_EINVAL, "stores must be 0, 1 or 2");
    if (cfg->pair_offset < 0 || cfg->pair_offset % 4 != 0 || cfg->pair_offset + cfg->n_pairs > ((int64_t)1 << 34))
        return fail(nullptr, MCINV_EINVAL, "pair_offset must be a non-negative multiple of 4 (pairs below 2^34)");
    const int64_t P = cfg->n_pairs, G = cfg->n_groups;
    if (G < 1 || P % G != 0) return fail(nullptr, MCINV_EINVAL, "n_groups must divide n_pairs");
    const int64_t gs = P / G;
    if (G > 1) {
        const bool pow2 = (gs & (gs - 1)) == 0;
        if (gs % 4 != 0 || (gs <= 256 && !pow2) || (gs > 256 && gs % 256 != 0))
            return fail(nullptr, MCINV_EINVAL,
                        "pairs per group must be a power of two in [4, 256] or a multiple of 256");
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || cfg->device < 0 || cfg->device >= ndev)
        return fail(nullptr, MCINV_EDEVICE, "no such HIP device");

    // the owner destroys a partly built context on every early return or exception
    std::unique_ptr<mcinv_ctx, void (*)(mcinv_ctx*)> owner(new mcinv_ctx(), mcinv_destroy);
    mcinv_ctx* c = owner.get();
    c->cfg = *cfg;
    c->cplx = cfg->sweep_dtype == MCINV_C64 || cfg->sweep_dtype == MCINV_C128;
    c->comps = c->cplx ? 2 : 1;
    c->elem = elem_size(cfg->sweep_dtype);
    c->P = P;
    c->ld = (P + 3) / 4 * 4;
    c->G = G;
    c->gs = gs;
    const int64_t lanes = G == 1 ? kWave : std::min<int64_t>(gs / 4, kWave);
    int64_t sh = 0;
    while ((int64_t)1 << sh < lanes) ++sh;
    c->lg_shift = sh;
    c->pairs_per_col = lanes * kPairsPerLane;
    c->ntiles = (c->ld + kPairsPerWave - 1) / kPairsPerWave;
    c->cpt = kWave / lanes;
    c->A = c->ntiles * c->cpt;
    c->nslots = G >= 16 ? 1 : kSlotsSmallG;
    c->slot_len.assign(c->nslots, 0.0);

    auto bail = [&](mcinv_status s) {
        g_error = c->err;
        return s;
    };
    mcinv_status s = set_device(c);
    if (s != MCINV_OK) return bail(s);
    if (cfg->stream) {
        c->stream = (hipStream_t)cfg->stream;
    } else {
        if (hipStreamCreate(&c->stream) != hipSuccess) return bail(fail(c, MCINV_EDEVICE, "hipStreamCreate failed"));
        c->own_stream = true;
    }
    if ((s = dalloc(c, &c->d_flag, 1)) != MCINV_OK) return bail(s);
    if ((s = dalloc(c, &c->d_partial, 2 * 128)) != MCINV_OK) return bail(s);
    if ((s = dalloc(c, &c->d_counter, 1)) != MCINV_OK) return bail(s);
    if ((s = dalloc(c, &c->d_maxrel, 1)) != MCINV_OK) return bail(s);
    if ((s = dalloc(c, &c->d_geyer, 8)) != MCINV_OK) return bail(s);
    if ((s = dalloc(c, &c->d_slot_len, (size_t)c->nslots)) != MCINV_OK) return bail(s);
    if (hipMemsetAsync(c->d_flag, 0, sizeof(int32_t), c->stream) != hipSuccess ||
        hipMemsetAsync(c->d_counter, 0, sizeof(uint32_t), c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess)
        return bail(fail(c, MCINV_EDEVICE, "initial memset failed"));
    *out = owner.release();
    return MCINV_OK;
} catch (...) {
    return mcinv::exception_status([&](mcinv_status s_, const std::string& m_) { fail(nullptr, s_, m_); });
}

void mcinv_destroy(mcinv_ctx* c)
{
    if (!c) return;
    (void)hipSetDevice(c->cfg.device);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    free_matrix(c);
    dfree(c->d_flag);
    dfree(c->d_partial);
    dfree(c->d_counter);
    dfree(c->d_maxrel);
    dfree(c->d_geyer);
    dfree(c->d_slot_len);
    for (hipEvent_t e : c->events) (void)hipEventDestroy(e);
    if (c->side) (void)hipStreamDestroy(c->side);
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

mcinv_status mcinv_load_csr(mcinv_ctx* c, int64_t n, int64_t nnz, const int64_t* row_ptr, const int32_t* col_idx,
                            const void* values, int32_t value_dtype)
try {
    if (!c) return fail(nullptr, MCINV_EINVAL, "null context");
    MC_TRY(set_device(c));
    if (value_dtype != MCINV_R64 && value_dtype != MCINV_C128)
        return fail(c, MCINV_EINVAL, "values must be float64 (MCINV_R64) or complex128 (MCINV_C128)");
    if (value_dtype == MCINV_C128 && !c->cplx)
        return fail(c, MCINV_EINVAL, "a complex matrix needs a complex sweep dtype");
    Prepared h;
    bool singular = false;
    const std::string why = prepare_matrix(n, nnz, row_ptr, col_idx, (const double*)values,
                                           value_dtype == MCINV_C128, h, &singular);
    if (!why.empty()) return fail(c, singular ? MCINV_ESINGULAR : MCINV_EINVAL, why);
    if (c->cfg.hermitian) {
        // w = z needs c_ji = conj(c_ij) (then v = u exactly) and a positive real
        // diagonal (then b = a).
        for (int64_t q = 0; q < n; ++q)
            if (!(h.diag[q].imag() == 0.0 && h.diag[q].real() > 0.0))
                return fail(c, MCINV_EINVAL, "hermitian mode needs a positive real diagonal");
        for (const MergedEntry& e : h.ent)
            if (!(e.u == e.v)) return fail(c, MCINV_EINVAL, "hermitian mode: the matrix is not hermitian");
    }
    const bool real_values = value_dtype == MCINV_R64;
    const int32_t ncolors = h.ncolors;
    const std::vector<int64_t>& color_ptr = h.color_ptr;

    free_matrix(c);
    c->n = n;
    c->nnz = nnz;
    c->n_off = (int64_t)h.ent.size();
    c->ncolors = ncolors;
    c->perm = h.perm;
    c->pos = h.pos;
    c->color = h.color;
    c->color_ptr = h.color_ptr;
    c->real_values = real_values;
    {
        // the values a restored chain continues under: coefficients and scales
        uint64_t vh = kFnvBasis;
        for (const MergedEntry& e : h.ent) {
            vh = fnv1a(vh, &e.col, sizeof(e.col));
            vh = fnv1a(vh, &e.u, sizeof(e.u));
            vh = fnv1a(vh, &e.v, sizeof(e.v));
        }
        for (size_t q = 0; q < h.a.size(); ++q) {
            vh = fnv1a(vh, &h.a[q], sizeof(h.a[q]));
            vh = fnv1a(vh, &h.b[q], sizeof(h.b[q]));
            vh = fnv1a(vh, &h.diag[q], sizeof(h.diag[q]));
        }
        c->value_hash = vh;
    }
    c->q_hash = 0;
    c->tpart_off.assign(ncolors + 1, 0);
    for (int32_t k = 0; k < ncolors; ++k) {
        const int64_t rows = color_ptr[k + 1] - color_ptr[k];
        c->tpart_off[k + 1] = c->tpart_off[k] + (rows + 3) / 4 * c->ntiles;
    }
    c->npart = c->tpart_off[ncolors];
    // One pass over all tiles unless asked otherwise: on the pedigree and lattice
    // workloads, passes of one tile (a ~200 MB slice that could stay in the
    // Infinity Cache) measured slower than one launch per colour over all tiles.
    c->pass_tiles = c->cfg.pass_tiles > 0 ? c->cfg.pass_tiles : c->ntiles;

    mcinv_status s;
    switch (c->cfg.sweep_dtype) {
    case MCINV_R32: s = upload_matrix<float>(c, h); break;
    case MCINV_R64: s = upload_matrix<double>(c, h); break;
    case MCINV_C64: s = upload_matrix<Cx<float>>(c, h); break;
    default: s = upload_matrix<Cx<double>>(c, h); break;
    }
    if (s != MCINV_OK) return s;
    MC_TRY(upload(c, &c->d_perm, h.perm));
    const size_t state_bytes = (size_t)n * c->ld * c->elem;
    HIP_TRY(c, hipMalloc(&c->d_z, state_bytes));
    if (!c->cfg.hermitian) HIP_TRY(c, hipMalloc(&c->d_w, state_bytes));
    HIP_TRY(c, hipMemsetAsync(c->d_z, 0, state_bytes, c->stream));
    if (!c->cfg.hermitian) HIP_TRY(c, hipMemsetAsync(c->d_w, 0, state_bytes, c->stream));
    HIP_TRY(c, hipMemsetAsync(c->d_flag, 0, sizeof(int32_t), c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    c->sweeps = 0;
    c->samples = 0;
    c->batch_len = 1;
    c->slot_len.assign(c->nslots, 0.0);
    c->loaded = true;
    return MCINV_OK;
} catch (...) {
    return mcinv::exception_status([&](mcinv_status s_, const std::string& m_) { fail(c, s_, m_); });
}

mcinv_status mcinv_set_requested(mcinv_ctx* c, uint32_t flags, const int64_t* block_rows, int64_t n_block_rows,
                                 const int64_t* block_cols, int64_t n_block_cols, const int64_t* entry_i,
                                 const int64_t* entry_j, int64_t n_entries)
try {
    MC_TRY(check_ready(c));
    if (flags & ~(MCINV_REQ_DIAG | MCINV_REQ_TRACE | MCINV_REQ_BLOCK | MCINV_REQ_ENTRIES | MCINV_REQ_QTRACE))
        return fail(c, MCINV_EINVAL, "unknown request flag");
    if ((flags & MCINV_REQ_QTRACE) && c->q_nnz < 0)
        return fail(c, MCINV_ESTATE, "MCINV_REQ_QTRACE needs mcinv_set_trace_matrix first");
    const bool want_block = (flags & MCINV_REQ_BLOCK) && n_block_rows > 0 && n_block_cols > 0;
    const bool want_entries = (flags & MCINV_REQ_ENTRIES) && n_entries > 0;
    if (want_block && (!block_rows || !block_cols)) return fail(c, MCINV_EINVAL, "null block index arrays");
    if (want_entries && (!entry_i || !entry_j)) return fail(c, MCINV_EINVAL, "null entry arrays");
    auto to_pos = [&](const int64_t* idx, int64_t m, std::vector<int64_t>& out) -> bool {
        out.resize(m);
        for (int64_t k = 0; k < m; ++k) {
            if (idx[k] < 0 || idx[k] >= c->n) return false;
            out[k] = c->pos[idx[k]];
        }
        return true;
    };
    std::vector<int64_t> I, J, ei, ej;
    if (want_block && (!to_pos(block_rows, n_block_rows, I) || !to_pos(block_cols, n_block_cols, J)))
        return fail(c, MCINV_EINVAL, "block index out of range");
    if (want_entries && (!to_pos(entry_i, n_entries, ei) || !to_pos(entry_j, n_entries, ej)))
        return fail(c, MCINV_EINVAL, "entry index out of range");

    HIP_TRY(c, hipStreamSynchronize(c->stream));
    free_requests(c);
    c->flags = flags;
    c->nI = want_block ? n_block_rows : 0;
    c->nJ = want_block ? n_block_cols : 0;
    c->ne = want_entries ? n_entries : 0;
    if (!want_block) c->flags &= ~MCINV_REQ_BLOCK;
    if (!want_entries) c->flags &= ~MCINV_REQ_ENTRIES;
    MC_TRY(dalloc(c, &c->d_slot_len, (size_t)c->nslots));
    if (c->flags & MCINV_REQ_DIAG) {
        const size_t cnt = (size_t)(c->nslots * c->diag_slot_stride());
        MC_TRY(dalloc(c, &c->d_diag, cnt));
        HIP_TRY(c, hipMemsetAsync(c->d_diag, 0, cnt * sizeof(double), c->stream));
    }
    if (c->flags & MCINV_REQ_TRACE) {
        MC_TRY(dalloc(c, &c->d_tpart, (size_t)(c->npart * c->comps)));
        MC_TRY(grow_series(c, 4096));
    }
    if (c->flags & MCINV_REQ_QTRACE) {
        MC_TRY(dalloc(c, &c->d_qpart, (size_t)(qtrace_partials(c) * c->comps)));
        MC_TRY(grow_series(c, 4096, &c->d_qseries, &c->qseries_cap));
    }
    if (c->flags & MCINV_REQ_BLOCK) {
        MC_TRY(upload(c, &c->d_I, I));
        MC_TRY(upload(c, &c->d_J, J));
        const size_t cnt = (size_t)(c->nslots * c->block_slot_stride());
        MC_TRY(dalloc(c, &c->d_block, cnt));
        HIP_TRY(c, hipMemsetAsync(c->d_block, 0, cnt * sizeof(double), c->stream));
    }
    if (c->flags & MCINV_REQ_ENTRIES) {
        MC_TRY(upload(c, &c->d_ei, ei));
        MC_TRY(upload(c, &c->d_ej, ej));
        const size_t cnt = (size_t)(c->nslots * c->entry_slot_stride());
        MC_TRY(dalloc(c, &c->d_entries, cnt));
        HIP_TRY(c, hipMemsetAsync(c->d_entries, 0, cnt * sizeof(double), c->stream));
    }
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    c->samples = 0;
    c->batch_len = 1;
    c->slot_len.assign(c->nslots, 0.0);
    c->requested = true;
    return MCINV_OK;
} catch (...) {
    return mcinv::exception_status([&](mcinv_status s_, const std::string& m_) { fail(c, s_, m_); });
}

mcinv_status mcinv_burn_in(mcinv_ctx* c, int64_t sweeps)
try {
    MC_TRY(check_ready(c));
    if (sweeps < 0) return fail(c, MCINV_EINVAL, "negative sweep count");
    MC_TRY(dispatch_sweeps(c, sweeps, false));
    c->sweeps += sweeps;
    return check_flag(c);
} catch (...) {
    return mcinv::exception_status([&](mcinv_status s_, const std::string& m_) { fail(c, s_, m_); });
}

mcinv_status mcinv_tune_launch(mcinv_ctx* c, int32_t sweeps_per_trial, int32_t* xcd_order, double* ms_orders)
try {
    MC_TRY(check_ready(c));
    if (sweeps_per_trial < 1) return fail(c, MCINV_EINVAL, "sweeps_per_trial must be >= 1");
    hipEvent_t e0, e1;
    HIP_TRY(c, hipEventCreate(&e0));
    HIP_TRY(c, hipEventCreate(&e1));
    double ms[kLaunchOrders] = {};
    mcinv_status s = MCINV_OK;
    for (int order = 0; order < kLaunchOrders && s == MCINV_OK; ++order) {
        c->cfg.xcd_order = order;
        // every sweep draws its own noise (counter = sweep index), as in burn-in
        if ((s = dispatch_sweeps(c, 1, false)) != MCINV_OK) break;
        c->sweeps += 1;
        if (hipEventRecord(e0, c->stream) != hipSuccess) s = fail(c, MCINV_EDEVICE, "hipEventRecord failed");
        if (s == MCINV_OK) s = dispatch_sweeps(c, sweeps_per_trial, false);
        if (s == MCINV_OK) c->sweeps += sweeps_per_trial;
        float t = 0.f;
        if (s == MCINV_OK && (hipEventRecord(e1, c->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                              hipEventElapsedTime(&t, e0, e1) != hipSuccess))
            s = fail(c, MCINV_EDEVICE, "timing the launch orders failed");
        ms[order] = (double)t / sweeps_per_trial;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (s != MCINV_OK) return s;
    int best = 0;
    for (int order = 1; order < kLaunchOrders; ++order)
        if (ms[order] < ms[best]) best = order;
    c->cfg.xcd_order = best;
    if (xcd_order) *xcd_order = best;
    if (ms_orders)
        for (int order = 0; order < kLaunchOrders; ++order) ms_orders[order] = ms[order];
    return check_flag(c);
} catch (...) {
    return mcinv::exception_status([&](mcinv_status s_, const std::string& m_) { fail(c, s_, m_); });
}

mcinv_status mcinv_sample(mcinv_ctx* c, int64_t sweeps)
try {
    MC_TRY(check_ready(c));
    if (!c->requested) return fail(c, MCINV_ESTATE, "call mcinv_set_requested before sampling");
    if (sweeps < 0) return fail(c, MCINV_EINVAL, "negative sweep count");
    MC_TRY(dispatch_sweeps(c, sweeps, true));
    c->sweeps += sweeps;
    return check_flag(c);
} catch (...) {
    return mcinv::exception_status([&](mcinv_status s_, const std::string& m_) { fail(c, s_, m_); });
}

mcinv_status mcinv_sample_until(mcinv_ctx* c, double rel_se, int64_t max_sweeps, int64_t check_every,
                                int64_t* sweeps_done, double* achieved)
try {
    constexpr int64_t kMinBatchLen = 16;
    MC_TRY(check_ready(c));
    if (!c->requested || !(c->flags & MCINV_REQ_DIAG))
        return fail(c, MCINV_ESTATE, "sample_until needs MCINV_REQ_DIAG requested");
    if (check_every < 1 || max_sweeps < 0) return fail(c, MCINV_EINVAL, "bad sweep counts");
    int64_t done = 0;
    double maxrel = INFINITY;
    while (done < max_sweeps) {
        const int64_t chunk = std::min(check_every, max_sweeps - done);
        MC_TRY(dispatch_sweeps(c, chunk, true));
        c->sweeps += chunk;
        done += chunk;
        MC_TRY(finalize_diag(c, true));
        unsigned long long bits = 0;
        HIP_TRY(c, hipMemcpyAsync(&bits, c->d_maxrel, sizeof(bits), hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        std::memcpy(&maxrel, &bits, sizeof(double));
        MC_TRY(check_flag(c));
        // with fewer than 16 groups the SE clusters include time batches, which
        // must be long against the chains' autocorrelation to be independent
        const bool batches_ok = c->nslots == 1 || c->batch_len >= kMinBatchLen;
        if (maxrel <= rel_se && batches_ok) break;
    }
    if (sweeps_done) *sweeps_done = done;
    if (achieved) *achieved = maxrel;
    return MCINV_OK;
} catch (...) {
    return mcinv::exception_status([&](mcinv_status s_, const std::string& m_) { fail(c, s_, m_); });
}

mcinv_status mcinv_sample_until_trace(mcinv_ctx* c, double rel_se, int64_t max_sweeps, int64_t check_every,
                                      int64_t* sweeps_done, double* achieved)
try {
    constexpr double kMinEffectiveSamples = 50.0;
    MC_TRY(check_ready(c));
    if (!c->requested || !(c->flags & (MCINV_REQ_TRACE | MCINV_REQ_QTRACE)))
        return fail(c, MCINV_ESTATE, "sample_until_trace needs MCINV_REQ_TRACE or MCINV_REQ_QTRACE requested");
    const bool use_q = (c->flags & MCINV_REQ_QTRACE) != 0;
    if (check_every < 1 || max_sweeps < 0) return fail(c, MCINV_EINVAL, "bad sweep counts");
    int64_t done = 0;
    double rel = INFINITY;
    while (done < max_sweeps) {
        const int64_t chunk = std::min(check_every, max_sweeps - done);
        MC_TRY(dispatch_sweeps(c, chunk, true));
        c->sweeps += chunk;
        done += chunk;
        MC_TRY(check_flag(c));
        HIP_TRY(c, launch_geyer(use_q ? c->d_qseries : c->d_series, c->samples, c->comps, 1.0 / (double)c->P,
                                c->d_geyer, c->stream));
        double g[6];
        HIP_TRY(c, hipMemcpyAsync(g, c->d_geyer, sizeof(g), hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        const double mag = std::sqrt(g[0] * g[0] + (c->comps == 2 ? g[1] * g[1] : 0.0));
        rel = g[5] / mag;
        if (!(rel >= 0.0)) rel = INFINITY;
        // Geyer's SE is trusted only on a series of at least kMinEffectiveSamples
        // effective samples (N_eff = S gamma_0 / sigma^2): shorter series give
        // too small an error (the truncated autocovariance sum is short)
        if (rel <= rel_se && (g[4] >= kMinEffectiveSamples || !(g[3] > 0.0))) break;  // sigma^2 = 0: exact
    }
    if (sweeps_done) *sweeps_done = done;
    if (achieved) *achieved = rel;
    return MCINV_OK;
} catch (...) {
    return mcinv::exception_status([&](mcinv_status s_, const std::string& m_) { fail(c, s_, m_); });
}

mcinv_status mcinv_read_estimates(mcinv_ctx* c, uint32_t quantity, double* est, double* stderr_, int64_t capacity)
try {
    MC_TRY(check_ready(c));
    if (!c->requested || !(c->flags & quantity)) return fail(c, MCINV_ESTATE, "quantity was not requested");
    int64_t M = 0;
    if (quantity == MCINV_REQ_DIAG) {
        M = c->n;
        if (capacity < M) return fail(c, MCINV_EINVAL, "capacity too small");
        MC_TRY(finalize_diag(c, false));
    } else if (quantity == MCINV_REQ_BLOCK) {
        M = c->nI * c->nJ;
        if (capacity < M) return fail(c, MCINV_EINVAL, "capacity too small");
        MC_TRY(finalize_flat(c, c->d_block, M, c->block_slot_stride()));
    } else if (quantity == MCINV_REQ_ENTRIES) {
        M = c->ne;
        if (capacity < M) return fail(c, MCINV_EINVAL, "capacity too small");
        MC_TRY(finalize_flat(c, c->d_entries, M, c->entry_slot_stride()));
    } else if (quantity == MCINV_REQ_TRACE || quantity == MCINV_REQ_QTRACE) {
        if (capacity < 1) return fail(c, MCINV_EINVAL, "capacity too small");
        if (c->samples < 1) return fail(c, MCINV_ESTATE, "no samples yet");
        const double* series = quantity == MCINV_REQ_TRACE ? c->d_series : c->d_qseries;
        HIP_TRY(c, launch_geyer(series, c->samples, c->comps, 1.0 / (double)c->P, c->d_geyer, c->stream));
        double g[6];
        HIP_TRY(c, hipMemcpyAsync(g, c->d_geyer, sizeof(g), hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        if (est) {
            est[0] = g[0];
            if (c->comps == 2) est[1] = g[1];
        }
        if (stderr_) stderr_[0] = g[5];
        return MCINV_OK;
    } else {
        return fail(c, MCINV_EINVAL, "quantity must be exactly one MCINV_REQ_* flag");
    }
    if (est)
        HIP_TRY(c, hipMemcpyAsync(est, c->d_est, sizeof(double) * M * c->comps, hipMemcpyDeviceToHost, c->stream));
    if (stderr_) HIP_TRY(c, hipMemcpyAsync(stderr_, c->d_se, sizeof(double) * M, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return MCINV_OK;
} catch (...) {
    return mcinv::exception_status([&](mcinv_status s_, const std::string& m_) { fail(c, s_, m_); });
}

mcinv_status mcinv_read_trace_stats(mcinv_ctx* c, uint32_t quantity, double* stats)
try {
    MC_TRY(check_ready(c));
    if (quantity != MCINV_REQ_TRACE && quantity != MCINV_REQ_QTRACE)
        return fail(c, MCINV_EINVAL, "quantity must be MCINV_REQ_TRACE or MCINV_REQ_QTRACE");
    if (!c->requested || !(c->flags & quantity)) return fail(c, MCINV_ESTATE, "quantity was not requested");
    if (!stats) return fail(c, MCINV_EINVAL, "null output");
    if (c->samples < 1) return fail(c, MCINV_ESTATE, "no samples yet");
    const double* series = quantity == MCINV_REQ_TRACE ? c->d_series : c->d_qseries;
    HIP_TRY(c, launch_geyer(series, c->samples, c->comps, 1.0 / (double)c->P, c->d_geyer, c->stream));
    double g[8];
    HIP_TRY(c, hipMemcpyAsync(g, c->d_geyer, sizeof(g), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    stats[0] = g[0];                 // mean, real part
    stats[1] = c->comps == 2 ? g[1] : 0.0;
    stats[2] = g[2];                 // gamma_0: variance of the per-sweep values
    stats[3] = g[3];                 // sigma^2 of the initial positive sequence
    stats[4] = g[4];                 // effective length S gamma_0 / sigma^2
    stats[5] = g[5];                 // standard error sqrt(sigma^2 / S)
    stats[6] = (double)c->samples;   // S
    stats[7] = g[6];                 // gamma_0 of the real part
    stats[8] = g[7];                 // gamma_0 of the imaginary part
    return MCINV_OK;
} catch (...) {
    return mcinv::exception_status([&](mcinv_status s_, const std::string& m_) { fail(c, s_, m_); });
}

mcinv_status mcinv_read_state(mcinv_ctx* c, int32_t which, void* host, int64_t bytes)
try {
    MC_TRY(check_ready(c));
    if (which != 0 && which != 1) return fail(c, MCINV_EINVAL, "which must be 0 (z) or 1 (w)");
    if (!host || bytes < c->n * c->P * (int64_t)c->elem) return fail(c, MCINV_EINVAL, "host buffer too small");
    std::vector<char> tmp((size_t)(c->n * c->ld * c->elem));
    HIP_TRY(c, hipMemcpyAsync(tmp.data(), which ? w_state(c) : c->d_z, tmp.size(), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    char* out = (char*)host;
    const size_t row_bytes = (size_t)c->P * c->elem;
    for (int64_t i = 0; i < c->n; ++i)
        std::memcpy(out + (size_t)i * row_bytes, tmp.data() + (size_t)c->pos[i] * c->ld * c->elem, row_bytes);
    return MCINV_OK;
} catch (...) {
    return mcinv::exception_status([&](mcinv_status s_, const std::string& m_) { fail(c, s_, m_); });
}

mcinv_status mcinv_write_state(mcinv_ctx* c, int32_t which, const void* host, int64_t bytes)
try {
    MC_TRY(check_ready(c));
    if (which != 0 && which != 1) return fail(c, MCINV_EINVAL, "which must be 0 (z) or 1 (w)");
    if (!host || bytes < c->n * c->P * (int64_t)c->elem) return fail(c, MCINV_EINVAL, "host buffer too small");
    if (which == 1 && c->cfg.hermitian) return fail(c, MCINV_EINVAL, "hermitian mode: w is z; write z");
    std::vector<char> tmp((size_t)(c->n * c->ld * c->elem), 0);
    const char* in = (const char*)host;
    const size_t row_bytes = (size_t)c->P * c->elem;
    for (int64_t i = 0; i < c->n; ++i)
        std::memcpy(tmp.data() + (size_t)c->pos[i] * c->ld * c->elem, in + (size_t)i * row_bytes, row_bytes);
    HIP_TRY(c, hipMemcpyAsync(which ? c->d_w : c->d_z, tmp.data(), tmp.size(), hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return MCINV_OK;
} catch (...) {
    return mcinv::exception_status([&](mcinv_status s_, const std::string& m_) { fail(c, s_, m_); });
}

}  // extern "C"

template <typename V>
static mcinv_status upload_q(mcinv_ctx* c, const std::vector<int64_t>& rp, const std::vector<int64_t>& col,
                             const std::vector<cd>& val)
{
    std::vector<V> v(val.size());
    for (size_t e = 0; e < val.size(); ++e) v[e] = cast_val<V>(val[e]);
    dfree(c->d_qrp);
    dfree(c->d_qcol);
    dfree(c->d_qval);
    MC_TRY(upload(c, &c->d_qrp, rp));
    MC_TRY(upload(c, &c->d_qcol, col));
    V* dv = nullptr;
    MC_TRY(dalloc(c, &dv, std::max<size_t>(v.size(), 1)));
    if (!v.empty()) HIP_TRY(c, hipMemcpy(dv, v.data(), sizeof(V) * v.size(), hipMemcpyHostToDevice));
    c->d_qval = dv;
    return MCINV_OK;
}

extern "C" {

mcinv_status mcinv_set_trace_matrix(mcinv_ctx* c, int64_t nnz, const int64_t* row_ptr, const int32_t* col_idx,
                                    const void* values, int32_t value_dtype)
try {
    MC_TRY(check_ready(c));
    if (c->requested && (c->flags & MCINV_REQ_QTRACE))
        return fail(c, MCINV_ESTATE, "Q cannot change while MCINV_REQ_QTRACE is requested");
    if (value_dtype != MCINV_R64 && value_dtype != MCINV_C128)
        return fail(c, MCINV_EINVAL, "Q values must be float64 or complex128");
    if (value_dtype == MCINV_C128 && !c->cplx) return fail(c, MCINV_EINVAL, "a complex Q needs a complex sweep dtype");
    if (nnz < 0 || !row_ptr || (nnz > 0 && (!col_idx || !values))) return fail(c, MCINV_EINVAL, "bad Q arrays");
    const int64_t n = c->n;
    if (row_ptr[0] != 0 || row_ptr[n] != nnz) return fail(c, MCINV_EINVAL, "Q row_ptr[0] must be 0, row_ptr[n] nnz");
    for (int64_t i = 0; i < n; ++i) {
        if (row_ptr[i + 1] < row_ptr[i]) return fail(c, MCINV_EINVAL, "Q row_ptr is decreasing");
        for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e)
            if (col_idx[e] < 0 || col_idx[e] >= n) return fail(c, MCINV_EINVAL, "Q column out of range");
    }
    const double* vd = (const double*)values;
    std::vector<int64_t> rp(n + 1, 0), col;
    std::vector<cd> val;
    col.reserve(nnz);
    val.reserve(nnz);
    for (int64_t q = 0; q < n; ++q) {
        const int64_t i = c->perm[q];
        for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
            col.push_back(c->pos[col_idx[e]]);
            val.push_back(value_dtype == MCINV_C128 ? cd(vd[2 * e], vd[2 * e + 1]) : cd(vd[e], 0.0));
        }
        rp[q + 1] = (int64_t)col.size();
    }
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    switch (c->cfg.sweep_dtype) {
    case MCINV_R32: MC_TRY(upload_q<float>(c, rp, col, val)); break;
    case MCINV_R64: MC_TRY(upload_q<double>(c, rp, col, val)); break;
    case MCINV_C64: MC_TRY(upload_q<Cx<float>>(c, rp, col, val)); break;
    default: MC_TRY(upload_q<Cx<double>>(c, rp, col, val)); break;
    }
    c->q_nnz = nnz;
    uint64_t qh = kFnvBasis;
    qh = fnv1a(qh, rp.data(), sizeof(int64_t) * rp.size());
    qh = fnv1a(qh, col.data(), sizeof(int64_t) * col.size());
    qh = fnv1a(qh, val.data(), sizeof(cd) * val.size());
    c->q_hash = qh;
    return MCINV_OK;
} catch (...) {
    return mcinv::exception_status([&](mcinv_status s_, const std::string& m_) { fail(c, s_, m_); });
}

mcinv_status mcinv_set_stop_rows(mcinv_ctx* c, const int64_t* rows, int64_t count)
try {
    MC_TRY(check_ready(c));
    if (count < 0 || (count > 0 && !rows)) return fail(c, MCINV_EINVAL, "bad stop-row list");
    std::vector<uint8_t> mask;
    if (count > 0) {
        mask.assign(c->n, 0);
        for (int64_t k = 0; k < count; ++k) {
            if (rows[k] < 0 || rows[k] >= c->n) return fail(c, MCINV_EINVAL, "stop row out of range");
            mask[rows[k]] = 1;
        }
    }
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    dfree(c->d_stop);
    if (count > 0) MC_TRY(upload(c, &c->d_stop, mask));
    return MCINV_OK;
} catch (...) {
    return mcinv::exception_status([&](mcinv_status s_, const std::string& m_) { fail(c, s_, m_); });
}

// ------------------------------------------------------------ checkpoint --
// File layout (native byte order): CkptHeader, slot_len[nslots], the request
// lists (I, J, entry i, entry j as positions), z, w (absent in hermitian
// mode), the diagonal / block / entry accumulators that are requested, the
// trace series and the Q-trace series (samples x comps each, when requested).
struct CkptHeader {
    char magic[8];
    int64_t version, n, nnz, n_off, P, ld, G, dtype, hermitian, noise, stream_id;
    uint64_t seed, fingerprint;
    int64_t flags, nI, nJ, ne, sweeps, samples, batch_len, nslots, q_nnz, requested, pair_offset;
};

}  // extern "C"

// The matrix a checkpoint belongs to: pattern sizes, colour order, the
// prepared coefficients and scales (a same-pattern matrix with other values
// must not continue the chains), and Q when the Q trace is accumulated.
static uint64_t fingerprint(const mcinv_ctx* c, bool with_q)
{
    uint64_t h = kFnvBasis;
    auto mix = [&](int64_t v) {
        for (int b = 0; b < 8; ++b) {
            h ^= (uint64_t)((v >> (8 * b)) & 0xff);
            h *= 1099511628211ull;
        }
    };
    mix(c->n);
    mix(c->nnz);
    mix(c->n_off);
    for (int64_t v : c->perm) mix(v);
    for (int64_t v : c->color_ptr) mix(v);
    mix((int64_t)c->value_hash);
    if (with_q) {
        mix(c->q_nnz);
        mix((int64_t)c->q_hash);
    }
    return h;
}

static bool write_all(FILE* f, const void* p, size_t bytes) { return bytes == 0 || fwrite(p, 1, bytes, f) == bytes; }
static bool read_all(FILE* f, void* p, size_t bytes) { return bytes == 0 || fread(p, 1, bytes, f) == bytes; }

// Device buffer <-> file through a host copy.
static mcinv_status dev_to_file(mcinv_ctx* c, FILE* f, const void* d, size_t bytes)
{
    if (bytes == 0) return MCINV_OK;
    std::vector<char> h(bytes);
    HIP_TRY(c, hipMemcpyAsync(h.data(), d, bytes, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (!write_all(f, h.data(), bytes)) return fail(c, MCINV_EINVAL, "checkpoint write failed");
    return MCINV_OK;
}

static mcinv_status file_to_dev(mcinv_ctx* c, FILE* f, void* d, size_t bytes)
{
    if (bytes == 0) return MCINV_OK;
    std::vector<char> h(bytes);
    if (!read_all(f, h.data(), bytes)) return fail(c, MCINV_EINVAL, "checkpoint file is truncated");
    HIP_TRY(c, hipMemcpyAsync(d, h.data(), bytes, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return MCINV_OK;
}

static mcinv_status save_body(mcinv_ctx* c, FILE* f)
{
    CkptHeader hd{};
    std::memcpy(hd.magic, "MCINVCK1", 8);
    hd.version = 3;
    hd.n = c->n;
    hd.nnz = c->nnz;
    hd.n_off = c->n_off;
    hd.P = c->P;
    hd.ld = c->ld;
    hd.G = c->G;
    hd.dtype = c->cfg.sweep_dtype;
    hd.hermitian = c->cfg.hermitian ? 1 : 0;
    hd.noise = c->cfg.noise;
    hd.stream_id = c->cfg.stream_id;
    hd.seed = c->cfg.seed;
    hd.pair_offset = c->cfg.pair_offset;
    hd.fingerprint = fingerprint(c, c->requested && (c->flags & MCINV_REQ_QTRACE));
    hd.flags = c->flags;
    hd.nI = c->nI;
    hd.nJ = c->nJ;
    hd.ne = c->ne;
    hd.sweeps = c->sweeps;
    hd.samples = c->samples;
    hd.batch_len = c->batch_len;
    hd.nslots = c->nslots;
    hd.q_nnz = c->q_nnz;
    hd.requested = c->requested ? 1 : 0;
    if (!write_all(f, &hd, sizeof(hd)) || !write_all(f, c->slot_len.data(), sizeof(double) * c->slot_len.size()))
        return fail(c, MCINV_EINVAL, "checkpoint write failed");
    MC_TRY(dev_to_file(c, f, c->d_I, sizeof(int64_t) * (size_t)c->nI));
    MC_TRY(dev_to_file(c, f, c->d_J, sizeof(int64_t) * (size_t)c->nJ));
    MC_TRY(dev_to_file(c, f, c->d_ei, sizeof(int64_t) * (size_t)c->ne));
    MC_TRY(dev_to_file(c, f, c->d_ej, sizeof(int64_t) * (size_t)c->ne));
    const size_t state = (size_t)c->n * c->ld * c->elem;
    MC_TRY(dev_to_file(c, f, c->d_z, state));
    if (!c->cfg.hermitian) MC_TRY(dev_to_file(c, f, c->d_w, state));
    if (c->requested) {
        if (c->flags & MCINV_REQ_DIAG)
            MC_TRY(dev_to_file(c, f, c->d_diag, sizeof(double) * (size_t)(c->nslots * c->diag_slot_stride())));
        if (c->flags & MCINV_REQ_BLOCK)
            MC_TRY(dev_to_file(c, f, c->d_block, sizeof(double) * (size_t)(c->nslots * c->block_slot_stride())));
        if (c->flags & MCINV_REQ_ENTRIES)
            MC_TRY(dev_to_file(c, f, c->d_entries, sizeof(double) * (size_t)(c->nslots * c->entry_slot_stride())));
        if (c->flags & MCINV_REQ_TRACE)
            MC_TRY(dev_to_file(c, f, c->d_series, sizeof(double) * (size_t)(c->samples * c->comps)));
        if (c->flags & MCINV_REQ_QTRACE)
            MC_TRY(dev_to_file(c, f, c->d_qseries, sizeof(double) * (size_t)(c->samples * c->comps)));
    }
    return MCINV_OK;
}

static mcinv_status restore_body(mcinv_ctx* c, FILE* f)
{
    CkptHeader hd{};
    if (!read_all(f, &hd, sizeof(hd)) || std::memcmp(hd.magic, "MCINVCK1", 8) != 0 || hd.version != 3)
        return fail(c, MCINV_EINVAL, "not an mcinv checkpoint");
    if (hd.n != c->n || hd.nnz != c->nnz || hd.n_off != c->n_off ||
        hd.fingerprint != fingerprint(c, hd.requested && (hd.flags & MCINV_REQ_QTRACE)))
        return fail(c, MCINV_EINVAL, "checkpoint was taken on a different matrix");
    if (hd.P != c->P || hd.G != c->G || hd.dtype != c->cfg.sweep_dtype || hd.hermitian != (c->cfg.hermitian ? 1 : 0) ||
        hd.noise != c->cfg.noise || hd.stream_id != (int64_t)c->cfg.stream_id || hd.seed != c->cfg.seed ||
        hd.nslots != c->nslots || hd.pair_offset != c->cfg.pair_offset)
        return fail(c, MCINV_EINVAL, "checkpoint was taken with a different configuration");
    if ((hd.flags & MCINV_REQ_QTRACE) && c->q_nnz != hd.q_nnz)
        return fail(c, MCINV_ESTATE, "set the same trace matrix Q before restoring");
    // Counts from the file size host buffers below: each must be non-negative
    // and its bytes must still be in the file, so a corrupt header fails here
    // instead of asking for a huge allocation.
    const long here = std::ftell(f);
    if (here < 0 || std::fseek(f, 0, SEEK_END) != 0) return fail(c, MCINV_EINVAL, "checkpoint file is not seekable");
    const long end = std::ftell(f);
    if (end < here || std::fseek(f, here, SEEK_SET) != 0) return fail(c, MCINV_EINVAL, "checkpoint file is not seekable");
    const int64_t words_left = (int64_t)(end - here) / 8;
    if (hd.nI < 0 || hd.nI > c->n || hd.nJ < 0 || hd.nJ > c->n || hd.ne < 0 || hd.ne > words_left ||
        hd.samples < 0 || hd.samples > hd.sweeps || hd.samples > words_left || hd.batch_len < 0 ||
        hd.nslots + hd.nI + hd.nJ + 2 * hd.ne > words_left)
        return fail(c, MCINV_EINVAL, "corrupt or truncated checkpoint (counts do not fit the file)");
    {
        // the exact size the header implies, so that a damaged file fails
        // before anything in the context changes
        using i128 = __int128;
        const i128 comps = c->comps, slots = hd.nslots;
        i128 bytes = 8 * ((i128)hd.nslots + hd.nI + hd.nJ + 2 * (i128)hd.ne);
        bytes += (i128)c->n * c->ld * c->elem * (c->cfg.hermitian ? 1 : 2);
        if (hd.requested) {
            if (hd.flags & MCINV_REQ_DIAG) bytes += 8 * slots * c->diag_slot_stride();
            if (hd.flags & MCINV_REQ_BLOCK) bytes += 8 * slots * c->G * (i128)hd.nI * hd.nJ * comps;
            if (hd.flags & MCINV_REQ_ENTRIES) bytes += 8 * slots * c->G * (i128)hd.ne * comps;
            if (hd.flags & MCINV_REQ_TRACE) bytes += 8 * (i128)hd.samples * comps;
            if (hd.flags & MCINV_REQ_QTRACE) bytes += 8 * (i128)hd.samples * comps;
        }
        if (bytes != (i128)(end - here))
            return fail(c, MCINV_EINVAL, "corrupt or truncated checkpoint (size does not match its header)");
    }
    std::vector<double> slot_len((size_t)hd.nslots);
    if (!read_all(f, slot_len.data(), sizeof(double) * slot_len.size()))
        return fail(c, MCINV_EINVAL, "checkpoint file is truncated");
    std::vector<int64_t> I(hd.nI), J(hd.nJ), ei(hd.ne), ej(hd.ne);
    if (!read_all(f, I.data(), sizeof(int64_t) * I.size()) || !read_all(f, J.data(), sizeof(int64_t) * J.size()) ||
        !read_all(f, ei.data(), sizeof(int64_t) * ei.size()) || !read_all(f, ej.data(), sizeof(int64_t) * ej.size()))
        return fail(c, MCINV_EINVAL, "checkpoint file is truncated");
    for (auto* v : {&I, &J, &ei, &ej})
        for (int64_t& x : *v) {
            if (x < 0 || x >= c->n) return fail(c, MCINV_EINVAL, "corrupt checkpoint");
            x = c->perm[x];   // positions -> original indices
        }
    if (hd.requested) {
        MC_TRY(mcinv_set_requested(c, (uint32_t)hd.flags, I.data(), hd.nI, J.data(), hd.nJ, ei.data(), ej.data(),
                                   hd.ne));
    } else {
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        free_requests(c);
    }
    const size_t state = (size_t)c->n * c->ld * c->elem;
    MC_TRY(file_to_dev(c, f, c->d_z, state));
    if (!c->cfg.hermitian) MC_TRY(file_to_dev(c, f, c->d_w, state));
    if (hd.requested) {
        if (c->flags & MCINV_REQ_DIAG)
            MC_TRY(file_to_dev(c, f, c->d_diag, sizeof(double) * (size_t)(c->nslots * c->diag_slot_stride())));
        if (c->flags & MCINV_REQ_BLOCK)
            MC_TRY(file_to_dev(c, f, c->d_block, sizeof(double) * (size_t)(c->nslots * c->block_slot_stride())));
        if (c->flags & MCINV_REQ_ENTRIES)
            MC_TRY(file_to_dev(c, f, c->d_entries, sizeof(double) * (size_t)(c->nslots * c->entry_slot_stride())));
        if (c->flags & MCINV_REQ_TRACE) {
            MC_TRY(grow_series(c, std::max<int64_t>(hd.samples, 1)));
            MC_TRY(file_to_dev(c, f, c->d_series, sizeof(double) * (size_t)(hd.samples * c->comps)));
        }
        if (c->flags & MCINV_REQ_QTRACE) {
            MC_TRY(grow_series(c, std::max<int64_t>(hd.samples, 1), &c->d_qseries, &c->qseries_cap));
            MC_TRY(file_to_dev(c, f, c->d_qseries, sizeof(double) * (size_t)(hd.samples * c->comps)));
        }
    }
    c->sweeps = hd.sweeps;
    c->samples = hd.samples;
    c->batch_len = hd.batch_len;
    c->slot_len = slot_len;
    HIP_TRY(c, hipMemsetAsync(c->d_flag, 0, sizeof(int32_t), c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return MCINV_OK;
}

extern "C" {

mcinv_status mcinv_save(mcinv_ctx* c, const char* path)
try {
    MC_TRY(check_ready(c));
    if (!path) return fail(c, MCINV_EINVAL, "null path");
    FILE* f = std::fopen(path, "wb");
    if (!f) return fail(c, MCINV_EINVAL, std::string("cannot open ") + path + " for writing");
    const mcinv_status s = save_body(c, f);
    if (std::fclose(f) != 0 && s == MCINV_OK) return fail(c, MCINV_EINVAL, "checkpoint write failed");
    return s;
} catch (...) {
    return mcinv::exception_status([&](mcinv_status s_, const std::string& m_) { fail(c, s_, m_); });
}

mcinv_status mcinv_restore(mcinv_ctx* c, const char* path)
try {
    MC_TRY(check_ready(c));
    if (!path) return fail(c, MCINV_EINVAL, "null path");
    FILE* f = std::fopen(path, "rb");
    if (!f) return fail(c, MCINV_EINVAL, std::string("cannot open ") + path);
    const mcinv_status s = restore_body(c, f);
    std::fclose(f);
    return s;
} catch (...) {
    return mcinv::exception_status([&](mcinv_status s_, const std::string& m_) { fail(c, s_, m_); });
}

mcinv_status mcinv_get_permutation(mcinv_ctx* c, int64_t* perm, int32_t* color_of_row)
try {
    MC_TRY(check_ready(c));
    if (perm) std::memcpy(perm, c->perm.data(), sizeof(int64_t) * c->n);
    if (color_of_row) std::memcpy(color_of_row, c->color.data(), sizeof(int32_t) * c->n);
    return MCINV_OK;
} catch (...) {
    return mcinv::exception_status([&](mcinv_status s_, const std::string& m_) { fail(c, s_, m_); });
}

// The difference of two coupled paths (same noise, starts 0 and x*_i = i,
// 1-based original index: Algorithm 1, step 1) obeys eq 12: noiseless
// Gauss-Seidel sweeps on C d = 0 (z) and C^dagger d = 0 (w), the same for
// every chain pair.  Allocates the two [n][ld] difference chains holding x*.
static mcinv_status coupled_start(mcinv_ctx* c, int64_t ld, void** zc, void** wc, int32_t** fl)
{
    const size_t bytes = (size_t)c->n * ld * c->elem;
    *zc = *wc = nullptr;
    *fl = nullptr;
    HIP_TRY(c, hipMalloc(zc, bytes));
    HIP_TRY(c, hipMalloc(wc, bytes));
    HIP_TRY(c, hipMalloc((void**)fl, sizeof(int32_t)));
    HIP_TRY(c, hipMemsetAsync(*fl, 0, sizeof(int32_t), c->stream));
    std::vector<char> init(bytes, 0);
    for (int64_t q = 0; q < c->n; ++q)
        for (int64_t p = 0; p < ld; ++p) {
            const double x = (double)(c->perm[q] + 1);
            char* dst = init.data() + ((size_t)q * ld + p) * c->elem;
            if (c->cfg.sweep_dtype == MCINV_R32 || c->cfg.sweep_dtype == MCINV_C64) {
                const float xf = (float)x;
                std::memcpy(dst, &xf, sizeof(float));
            } else {
                std::memcpy(dst, &x, sizeof(double));
            }
        }
    HIP_TRY(c, hipMemcpyAsync(*zc, init.data(), bytes, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(*wc, init.data(), bytes, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return MCINV_OK;
}

static mcinv_status noiseless_sweeps(mcinv_ctx* c, int64_t k, void* zc, void* wc, int64_t ld, int32_t* fl)
{
    if (c->cfg.hermitian) wc = zc;   // C^dagger = C: the w difference is the z difference
    switch (c->cfg.sweep_dtype) {
    case MCINV_R32: return run_sweeps<float>(c, k, false, (float*)zc, (float*)wc, ld, 1, MCINV_NOISE_NONE, fl, false);
    case MCINV_R64: return run_sweeps<double>(c, k, false, (double*)zc, (double*)wc, ld, 1, MCINV_NOISE_NONE, fl, false);
    case MCINV_C64:
        return run_sweeps<Cx<float>>(c, k, false, (Cx<float>*)zc, (Cx<float>*)wc, ld, 1, MCINV_NOISE_NONE, fl, false);
    default:
        return run_sweeps<Cx<double>>(c, k, false, (Cx<double>*)zc, (Cx<double>*)wc, ld, 1, MCINV_NOISE_NONE, fl,
                                      false);
    }
}

static mcinv_status max_abs(mcinv_ctx* c, const void* x, int64_t ld, unsigned long long* out, hipStream_t st)
{
    switch (c->cfg.sweep_dtype) {
    case MCINV_R32: HIP_TRY(c, launch_max_abs<float>((const float*)x, c->n, ld, out, st)); break;
    case MCINV_R64: HIP_TRY(c, launch_max_abs<double>((const double*)x, c->n, ld, out, st)); break;
    case MCINV_C64: HIP_TRY(c, launch_max_abs<Cx<float>>((const Cx<float>*)x, c->n, ld, out, st)); break;
    default: HIP_TRY(c, launch_max_abs<Cx<double>>((const Cx<double>*)x, c->n, ld, out, st)); break;
    }
    return MCINV_OK;
}

}  // extern "C"

template <typename V>
static mcinv_status coupling_sweep(mcinv_ctx* c, void* dz, void* dw, hipStream_t st)
{
    for (int32_t col = 0; col < c->ncolors; ++col)
        HIP_TRY(c, launch_coupling_sweep<V>(c->d_rows, (const Entry<V>*)c->d_ent, c->color_ptr[col],
                                            c->color_ptr[col + 1], c->cfg.hermitian != 0, (V*)dz, (V*)dw, st));
    return MCINV_OK;
}

static mcinv_status coupling_sweep_any(mcinv_ctx* c, void* dz, void* dw, hipStream_t st)
{
    switch (c->cfg.sweep_dtype) {
    case MCINV_R32: return coupling_sweep<float>(c, dz, dw, st);
    case MCINV_R64: return coupling_sweep<double>(c, dz, dw, st);
    case MCINV_C64: return coupling_sweep<Cx<float>>(c, dz, dw, st);
    default: return coupling_sweep<Cx<double>>(c, dz, dw, st);
    }
}

extern "C" {

mcinv_status mcinv_burn_in_coupled(mcinv_ctx* c, double tol, int64_t max_sweeps, int64_t* sweeps_done,
                                   double* diff_z, double* diff_w)
try {
    MC_TRY(check_ready(c));
    if (!(tol > 0.0) || max_sweeps < 0) return fail(c, MCINV_EINVAL, "tol must be > 0 and max_sweeps >= 0");
    // one difference value per row (ld = 1): x*_i - 0 with x*_i = i, 1-based
    void *dz = nullptr, *dw = nullptr;
    int32_t* fl = nullptr;
    unsigned long long* dmax = nullptr;
    mcinv_status s = coupled_start(c, 1, &dz, &dw, &fl);
    if (s == MCINV_OK && hipMalloc((void**)&dmax, 2 * sizeof(unsigned long long)) != hipSuccess)
        s = fail(c, MCINV_ENOMEM, "device allocation failed");
    void* dw_eff = c->cfg.hermitian ? dz : dw;  // C^dagger = C: the w difference is the z difference
    if (s == MCINV_OK && !c->side && hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking) != hipSuccess) {
        c->side = nullptr;
        s = fail(c, MCINV_EDEVICE, "hipStreamCreateWithFlags failed");
    }
    // The difference iteration runs on the side stream, ahead of the chains:
    // chain sweep k is issued on the context's stream once the difference
    // after k - 1 steps is still above tol (so that N >= k), and runs while the
    // next difference steps are checked.  The difference touches only the
    // matrix and its own buffers, so the two streams share nothing that either
    // writes; every chain sweep issued here is one of the N.
    int64_t N = 0;
    double dzm = INFINITY, dwm = INFINITY;
    for (int64_t k = 1; k <= max_sweeps && s == MCINV_OK; ++k) {
        if ((s = dispatch_sweeps(c, 1, false)) != MCINV_OK) break;
        c->sweeps += 1;
        N = k;
        if ((s = coupling_sweep_any(c, dz, dw, c->side)) != MCINV_OK) break;
        if (hipMemsetAsync(dmax, 0, 2 * sizeof(unsigned long long), c->side) != hipSuccess) {
            s = fail(c, MCINV_EDEVICE, "hipMemsetAsync failed");
            break;
        }
        if ((s = max_abs(c, dz, 1, dmax, c->side)) != MCINV_OK || (s = max_abs(c, dw_eff, 1, dmax + 1, c->side)) != MCINV_OK)
            break;
        unsigned long long bits[2] = {0, 0};
        if (hipMemcpyAsync(bits, dmax, sizeof(bits), hipMemcpyDeviceToHost, c->side) != hipSuccess ||
            hipStreamSynchronize(c->side) != hipSuccess) {
            s = fail(c, MCINV_EDEVICE, "copying the coupling difference failed");
            break;
        }
        std::memcpy(&dzm, &bits[0], sizeof(double));
        std::memcpy(&dwm, &bits[1], sizeof(double));
        if (!std::isfinite(dzm) || !std::isfinite(dwm)) {
            s = fail(c, MCINV_EDIVERGED, "coupled paths diverge: the Gauss-Seidel iteration of eq 12 does not "
                                         "contract (sp(T) or sp(S) >= 1)");
            break;
        }
        if (dzm < tol && dwm < tol) break;
    }
    if (c->side) (void)hipStreamSynchronize(c->side);
    (void)hipFree(dz);
    (void)hipFree(dw);
    (void)hipFree(fl);
    (void)hipFree(dmax);
    if (s != MCINV_OK) return s;
    if (sweeps_done) *sweeps_done = N;
    if (diff_z) *diff_z = dzm;
    if (diff_w) *diff_w = dwm;
    return check_flag(c);
} catch (...) {
    return mcinv::exception_status([&](mcinv_status s_, const std::string& m_) { fail(c, s_, m_); });
}

mcinv_status mcinv_check_convergence(mcinv_ctx* c, int64_t iters, double* rho_T, double* rho_S)
try {
    MC_TRY(check_ready(c));
    if (iters < 2) return fail(c, MCINV_EINVAL, "iters must be >= 2");
    const int64_t ld = 4;
    const size_t bytes = (size_t)c->n * ld * c->elem;
    void *zc = nullptr, *wc = nullptr;
    int32_t* fl = nullptr;
    {
        const mcinv_status s0 = coupled_start(c, ld, &zc, &wc, &fl);
        if (s0 != MCINV_OK) {
            (void)hipFree(zc);
            (void)hipFree(wc);
            (void)hipFree(fl);
            return s0;
        }
    }
    std::vector<char> host(bytes);
    auto norms = [&](double* nz, double* nw) -> mcinv_status {
        double m[2] = {0.0, 0.0};
        for (int which = 0; which < 2; ++which) {
            const void* src = which && !c->cfg.hermitian ? wc : zc;
            HIP_TRY(c, hipMemcpyAsync(host.data(), src, bytes, hipMemcpyDeviceToHost, c->stream));
            HIP_TRY(c, hipStreamSynchronize(c->stream));
            const int comps = c->comps;
            const bool f32 = c->cfg.sweep_dtype == MCINV_R32 || c->cfg.sweep_dtype == MCINV_C64;
            for (int64_t q = 0; q < c->n; ++q) {
                double re = 0, im = 0;
                const char* src = host.data() + (size_t)q * ld * c->elem;
                if (f32) {
                    re = ((const float*)src)[0];
                    if (comps == 2) im = ((const float*)src)[1];
                } else {
                    re = ((const double*)src)[0];
                    if (comps == 2) im = ((const double*)src)[1];
                }
                m[which] = std::max(m[which], std::sqrt(re * re + im * im));
            }
        }
        *nz = m[0];
        *nw = m[1];
        return MCINV_OK;
    };
    const int64_t half = iters / 2;
    double z1 = 0, w1 = 0, z2 = 0, w2 = 0;
    mcinv_status s = MCINV_OK;
    auto sweep = [&](int64_t k) -> mcinv_status { return noiseless_sweeps(c, k, zc, wc, ld, fl); };
    if ((s = sweep(half)) == MCINV_OK && (s = norms(&z1, &w1)) == MCINV_OK && (s = sweep(iters - half)) == MCINV_OK)
        s = norms(&z2, &w2);
    (void)hipFree(zc);
    (void)hipFree(wc);
    (void)hipFree(fl);
    if (s != MCINV_OK) return s;
    const double m = (double)(iters - half);
    auto rate = [&](double a, double b) -> double {
        if (!(a > 0.0) || !(b > 0.0)) return 0.0;
        if (!std::isfinite(a) || !std::isfinite(b)) return INFINITY;
        return std::pow(b / a, 1.0 / m);
    };
    if (rho_T) *rho_T = rate(z1, z2);
    if (rho_S) *rho_S = rate(w1, w2);
    return MCINV_OK;
} catch (...) {
    return mcinv::exception_status([&](mcinv_status s_, const std::string& m_) { fail(c, s_, m_); });
}

mcinv_status mcinv_get_info(mcinv_ctx* c, mcinv_info* out)
try {
    if (!c || !out) return fail(c, MCINV_EINVAL, "null argument");
    std::memset(out, 0, sizeof(*out));
    out->n = c->n;
    out->nnz = c->nnz;
    out->n_pairs = c->P;
    out->ld = c->ld;
    out->n_colors = c->ncolors;
    out->n_groups = (int32_t)c->G;
    out->sweeps_done = c->sweeps;
    out->samples_done = c->samples;
    out->batch_len = c->nslots > 1 ? c->batch_len : c->samples;
    out->n_batches = c->nslots > 1 ? (c->samples + c->batch_len - 1) / c->batch_len : 1;
    out->offdiag_entries = c->n_off;
    out->sweep_kernel_ms = c->sweep_ms;
    out->sweep_kernel_launches = c->sweep_launches;
    out->moment_kernel_ms = c->moment_ms;
    out->moment_kernel_launches = c->moment_launches;
    return MCINV_OK;
} catch (...) {
    return mcinv::exception_status([&](mcinv_status s_, const std::string& m_) { fail(c, s_, m_); });
}

mcinv_status mcinv_reset_profile(mcinv_ctx* c)
try {
    if (!c) return fail(nullptr, MCINV_EINVAL, "null context");
    c->sweep_ms = c->moment_ms = 0.0;
    c->sweep_launches = c->moment_launches = 0;
    return MCINV_OK;
} catch (...) {
    return mcinv::exception_status([&](mcinv_status s_, const std::string& m_) { fail(c, s_, m_); });
}

mcinv_status mcinv_noise_values(int32_t device, uint64_t seed, uint32_t stream_id, int32_t noise, int32_t dtype,
                                int64_t count, const int64_t* row, const int64_t* sweep, const int64_t* pair,
                                double* out)
try {
    if (count < 0 || (count > 0 && (!row || !sweep || !pair || !out)))
        return fail(nullptr, MCINV_EINVAL, "bad arguments");
    if (dtype != MCINV_R32 && dtype != MCINV_R64) return fail(nullptr, MCINV_EINVAL, "dtype must be R32 or R64");
    if (noise < 0 || noise > 2) return fail(nullptr, MCINV_EINVAL, "unknown noise kind");
    if (count == 0) return MCINV_OK;
    HIP_TRY(nullptr, hipSetDevice(device));
    int64_t *dr = nullptr, *dk = nullptr, *dp = nullptr;
    double* dout = nullptr;
    const size_t b = sizeof(int64_t) * count;
    HIP_TRY(nullptr, hipMalloc((void**)&dr, b));
    HIP_TRY(nullptr, hipMalloc((void**)&dk, b));
    HIP_TRY(nullptr, hipMalloc((void**)&dp, b));
    HIP_TRY(nullptr, hipMalloc((void**)&dout, sizeof(double) * count));
    hipError_t e = hipMemcpy(dr, row, b, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(dk, sweep, b, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(dp, pair, b, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = launch_noise_values(dtype == MCINV_R64, seed, stream_id, noise, count, dr, dk, dp, dout, nullptr);
    if (e == hipSuccess) e = hipMemcpy(out, dout, sizeof(double) * count, hipMemcpyDeviceToHost);
    (void)hipFree(dr);
    (void)hipFree(dk);
    (void)hipFree(dp);
    (void)hipFree(dout);
    if (e != hipSuccess) return fail(nullptr, MCINV_EDEVICE, std::string("noise kernel: ") + hipGetErrorString(e));
    return MCINV_OK;
} catch (...) {
    return mcinv::exception_status([&](mcinv_status s_, const std::string& m_) { fail(nullptr, s_, m_); });
}

const char* mcinv_last_error(const mcinv_ctx* c)
{
    return c ? c->err.c_str() : g_error.c_str();
}

}  // extern "C"
