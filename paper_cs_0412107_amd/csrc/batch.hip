// Batched form: hundreds of matrices of uneven size, each with P chain pairs,
// swept together (Sec. 2 eqs 4-5 for every matrix; moments of eq 1/C) by one
// persistent launch per call or by a graph of phase launches; the autotuner
// keeps the faster (the phased graph, on the pedigree batches measured).
//
// Persistent schedule.  Work items are (sweep, colour, matrix, chunk of
// rows) plus, when sampling with a requested block, one block-moment item
// per (sweep, matrix).  Items
// are numbered sweep-major, then colour, then matrix, and workgroups take
// them in increasing order from a device counter (a few at a time).  A
// matrix's items of one phase may start only when all of its items of the
// previous phase (previous colour, or the previous sweep's last phase) are
// complete: a per-matrix completion counter, released after the item's
// stores and acquired before its loads (agent-scope fences: the L2 caches of
// the XCDs are not coherent with each other).  Every item's dependencies were
// handed out earlier, so the oldest unfinished item can always run; a wait
// that exceeds its bound sets an error flag and every workgroup exits.
//
// Phased schedule: the same item code with one launch per phase (see
// k_batch_rows).  Either way a row item first stages its rows' merged entries
// in LDS (batch_rows).
//
// Lane layout: a row's P pairs are spread over P/4 lanes (4 pairs each, one
// Philox block per lane); a wave holds 256/P rows.  The gather, noise and
// update arithmetic is the single-matrix kernel's, in the same order, so a
// batched matrix's chains are bit-identical to the same matrix swept alone.
#include "batch.h"
#include "device_common.h"
#include "mfma_tile.h"

#ifndef MCINV_GATHER_U4
#define MCINV_GATHER_U4 4
#endif

namespace mcinv {

struct alignas(16) Quad4 {
    float v[4];
};

// The rows of an item are consecutive positions, so their merged entries
// form one contiguous range; up to kBatchLdsEnt of them (16 KB) are staged in
// LDS once per item and every lane of a row reads its entries from there.
constexpr int kBatchLdsEnt = 1024;

// eb + (rr.begin - e0) is row rr's first entry (eb: the item's staged
// entries with e0 their first index, or the global array with e0 = 0)
__device__ inline void batch_rows_from(const BatchArgs& a, const BItem& it, int64_t sweep, int64_t sample,
                                       const Entry<float>* eb, int64_t e0)
{
    constexpr int U = MCINV_GATHER_U4;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int lpr = 1 << a.lane_shift;
    const int rpw = 64 >> a.lane_shift;
    const int lr = lane & (lpr - 1), rw = lane >> a.lane_shift;
    const int64_t p0 = (int64_t)lr * 4;
    const uint32_t stream = a.mats[it.m].stream;
    const int gs = a.P / a.G;
    const int lgb = gs / 4;  // lanes per group
    const int64_t slot = sample < 0 ? 0 : min(sample / a.batch_len, (int64_t)a.nslots_diag - 1);

    for (int64_t base = it.row_begin; base < it.row_end; base += 4 * rpw) {
        const int64_t q = base + wid * rpw + rw;
        if (q >= it.row_end) continue;  // whole rows (groups never span rows)
        const RowRec rr = a.rows[q];
        float az[4] = {0.f, 0.f, 0.f, 0.f}, aw[4] = {0.f, 0.f, 0.f, 0.f};
        const Entry<float>* e = eb + (rr.begin - e0);
        for (int b = 0; b < rr.count; b += U) {
            Quad4 xs[U], ys[U];
            float us[U], vs[U];
#pragma unroll
            for (int t = 0; t < U; ++t) {
                const bool ok = b + t < rr.count;
                const Entry<float> en = e[ok ? b + t : 0];
                us[t] = ok ? en.u : 0.f;
                vs[t] = ok ? en.v : 0.f;
                const int64_t off = (int64_t)en.col * a.P + p0;
                xs[t] = *reinterpret_cast<const Quad4*>(a.z + off);
                ys[t] = *reinterpret_cast<const Quad4*>(a.w + off);
            }
#pragma unroll
            for (int t = 0; t < U; ++t)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    az[j] = mul_add(us[t], xs[t].v[j], az[j]);
                    aw[j] = mul_add(vs[t], ys[t].v[j], aw[j]);
                }
        }
        float phi[4];
        noise4<float>(a.key0, a.key1, rr.orig, (uint32_t)sweep, (uint32_t)lr, stream, a.noise, phi);
        const Scales<float> s = a.sc[q];
        Quad4 zn, wn;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            zn.v[j] = noisy_update(s.a, phi[j], az[j]);
            wn.v[j] = noisy_update(s.b, phi[j], aw[j]);
        }
        *reinterpret_cast<Quad4*>(a.z + q * a.P + p0) = zn;
        *reinterpret_cast<Quad4*>(a.w + q * a.P + p0) = wn;
        float mag = 0.f;
#pragma unroll
        for (int j = 0; j < 4; ++j) mag = fmaxf(mag, fmaxf(fabsf(zn.v[j]), fabsf(wn.v[j])));
        if (!(mag < a.thresh)) atomicOr(a.flag, 1);

        if (sample >= 0 && a.diag != nullptr) {
            double pr = 0.0;
#pragma unroll
            for (int j = 0; j < 4; ++j) pr += (double)zn.v[j] * (double)wn.v[j];
            // lanes of one group are lgb consecutive lanes of this row
            for (int off = 1; off < lgb; off <<= 1) pr += __shfl_xor(pr, off);
            if ((lr & (lgb - 1)) == 0) a.diag[(slot * a.nrows + q) * a.G + lr / lgb] += pr;
        }
    }
}

// Called by every thread of the workgroup (the staging ends in a barrier);
// both schedules also separate consecutive items by a barrier, so the staged
// entries are not replaced while a wave still reads them.
__device__ inline void batch_rows(const BatchArgs& a, const BItem& it, int64_t sweep, int64_t sample)
{
    __shared__ Entry<float> s_ent[kBatchLdsEnt];
    if (it.row_end <= it.row_begin) return;   // no rows (the same for the whole workgroup)
    const int64_t e0 = a.rows[it.row_begin].begin;
    const RowRec last = a.rows[it.row_end - 1];
    const int64_t ne = last.begin + last.count - e0;
    if (ne <= kBatchLdsEnt) {
        for (int64_t k = threadIdx.x; k < ne; k += blockDim.x) s_ent[k] = a.ent[e0 + k];
        __syncthreads();
        batch_rows_from(a, it, sweep, sample, s_ent, e0);
    } else {
        batch_rows_from(a, it, sweep, sample, a.ent, 0);
    }
}

__device__ inline void batch_block(const BatchArgs& a, const BItem& it, int64_t sample)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int i16 = lane & 15, kg = lane >> 4;
    const int64_t slot = min(sample / a.batch_len, (int64_t)a.nslots_block - 1);
    const int bd = a.bdim;
    const int nt = (bd + 15) / 16;
    const int64_t* I = a.bI + a.mats[it.m].blk;
    const int64_t* J = a.bJ + a.mats[it.m].blk;
    double* acc_out = a.block + (slot * a.nmats + it.m) * (int64_t)bd * bd;
    for (int tt = wid; tt < nt * nt; tt += 4) {
        const int r0 = 16 * (tt / nt), t0 = 16 * (tt % nt);
        const int r = r0 + i16, c = t0 + i16;
        const bool zok = r < bd, wok = c < bd;
        const float* zrow = a.z + (zok ? I[r] : 0) * (int64_t)a.P;
        const float* wrow = a.w + (wok ? J[c] : 0) * (int64_t)a.P;
        f32x4 acc = f32x4{0.f, 0.f, 0.f, 0.f};
        bf16x3_tile16(zrow, zok, wrow, wok, 0, a.P, kg, acc);
        if (!wok) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int ro = r0 + 4 * kg + v;
            if (ro < bd) acc_out[(int64_t)ro * bd + c] += (double)acc[v];
        }
    }
}

__global__ __launch_bounds__(256) void k_batch(const BatchArgs a)
{
    __shared__ uint32_t s_first;
    __shared__ int s_stop;
    const int64_t sweep0 = a.clock->sweep;
    const int64_t sample0 = a.clock->sample;
    const int64_t total = a.nsweeps * a.items_per_sweep;

    if (threadIdx.x == 0) s_stop = 0;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) {
            s_first = atomicAdd(&a.clock->queue, (uint32_t)a.grab);
            if (__hip_atomic_load(&a.clock->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) s_stop = 1;
        }
        __syncthreads();
        const int64_t first = s_first;
        if (s_stop || first >= total) break;
        const int64_t last = first + a.grab < total ? first + a.grab : total;
        for (int64_t t = first; t < last; ++t) {
            const int64_t ls = t / a.items_per_sweep;
            const BItem it = a.items[t - ls * a.items_per_sweep];
            const uint32_t required = (uint32_t)(ls * a.mats[it.m].items_per_sweep + it.prior);
            if (threadIdx.x == 0) {
                uint32_t spins = 0;
                while (__hip_atomic_load(&a.done[it.m], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < required) {
                    if (++spins > a.spin_limit) {
                        __hip_atomic_store(&a.clock->error, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        s_stop = 1;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                }
            }
            __syncthreads();
            if (s_stop) break;
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            const int64_t sample = a.sample ? sample0 + ls : -1;
            if (it.kind == 0)
                batch_rows(a, it, sweep0 + ls, sample);
            else
                batch_block(a, it, sample);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            __syncthreads();
            if (threadIdx.x == 0) {
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
                __hip_atomic_fetch_add(&a.done[it.m], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        if (s_stop) break;
    }

    // The last workgroup to leave advances the clock and clears the counters
    // for the next launch (every other workgroup has finished).
    __syncthreads();
    if (threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        const uint32_t ticket = atomicAdd(&a.clock->exited, 1u);
        if (ticket == gridDim.x - 1) {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            for (int m = 0; m < a.nmats; ++m) a.done[m] = 0u;
            a.clock->queue = 0u;
            a.clock->exited = 0u;
            a.clock->sweep = sweep0 + a.nsweeps;
            if (a.sample) a.clock->sample = sample0 + a.nsweeps;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        }
    }
}

// Phased schedule: one launch per phase (a colour of every matrix, or the
// block moments of every matrix); kernel boundaries order the phases, so no
// fences are needed.  A one-thread kernel advances the clock after a sweep.
__global__ __launch_bounds__(256) void k_batch_rows(const BatchArgs a, const BItem* items)
{
    const BItem it = items[blockIdx.x];
    batch_rows(a, it, a.clock->sweep, a.sample ? a.clock->sample : -1);
}

__global__ __launch_bounds__(256) void k_batch_blocks(const BatchArgs a, const BItem* items)
{
    const BItem it = items[blockIdx.x];
    batch_block(a, it, a.clock->sample);
}

__global__ void k_batch_tick(BatchClock* clock, int32_t sample)
{
    if (threadIdx.x == 0) {
        clock->sweep += 1;
        if (sample) clock->sample += 1;
    }
}

hipError_t launch_batch_phase(const BatchArgs& a, const BItem* items, int64_t nitems, bool block_phase,
                              hipStream_t stream)
{
    if (nitems <= 0) return hipSuccess;
    if (block_phase)
        k_batch_blocks<<<dim3((unsigned)nitems), dim3(256), 0, stream>>>(a, items);
    else
        k_batch_rows<<<dim3((unsigned)nitems), dim3(256), 0, stream>>>(a, items);
    return hipGetLastError();
}

// Per matrix: max over its rows of |x[q * ld]| (lane 0), as double bits.
__global__ __launch_bounds__(256) void k_batch_max_abs(const float* x, int64_t nrows, int32_t ld,
                                                       const int32_t* row_mat, unsigned long long* out)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool ok = q < nrows;
    double v = ok ? fabs((double)x[q * ld]) : 0.0;
    if (!(v < __builtin_inf())) v = __builtin_inf();
    // rows of one matrix are contiguous: lanes whose matrix is the wave's
    // first one reduce across the wave first, the few others (a matrix
    // boundary inside the wave) go straight to memory
    const int32_t m = ok ? row_mat[q] : -1;
    const int32_t m0 = __shfl(m, 0);
    double r = (m == m0) ? v : 0.0;
    for (int off = 32; off > 0; off >>= 1) r = fmax(r, __shfl_xor(r, off));
    if ((threadIdx.x & 63) == 0 && m0 >= 0) atomicMax(out + m0, (unsigned long long)__double_as_longlong(r));
    if (ok && m != m0) atomicMax(out + m, (unsigned long long)__double_as_longlong(v));
}

hipError_t launch_batch_max_abs(const float* x, int64_t nrows, int32_t ld, const int32_t* row_mat,
                                unsigned long long* out, hipStream_t stream)
{
    if (nrows <= 0) return hipSuccess;
    k_batch_max_abs<<<dim3((unsigned)((nrows + 255) / 256)), dim3(256), 0, stream>>>(x, nrows, ld, row_mat, out);
    return hipGetLastError();
}

hipError_t launch_batch_tick(BatchClock* clock, bool sample, hipStream_t stream)
{
    k_batch_tick<<<dim3(1), dim3(64), 0, stream>>>(clock, sample ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_batch(const BatchArgs& a, int grid, hipStream_t stream)
{
    k_batch<<<dim3((unsigned)grid), dim3(256), 0, stream>>>(a);
    return hipGetLastError();
}

int batch_kernel_occupancy()
{
    int blocks = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, reinterpret_cast<const void*>(k_batch), 256, 0) !=
        hipSuccess)
        return 1;
    return blocks > 0 ? blocks : 1;
}

}  // namespace mcinv
