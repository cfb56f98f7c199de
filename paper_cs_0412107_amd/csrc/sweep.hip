// Colour sweep kernel: the coupled noisy Gauss-Seidel updates of eqs (4) and
// (5) for every row of one colour and every chain pair, with the diagonal and
// trace moments of eqs (1/C) and (tr) fused into the epilogue when sampling.
//
// Rows of one colour share no stored entry, so updating them in parallel is
// the same as updating them one after another: earlier colours already hold
// their sweep-k values and later colours their sweep k-1 values, exactly the
// j<i / j>i split of eqs (4)-(5) on the permuted matrix.
//
// Mapping (wave64): a wave owns one row and 256 consecutive chain pairs, four
// per lane.  The row's merged entries (column, z coefficient, w coefficient)
// are wave-uniform and arrive through scalar loads; each neighbour costs one
// coalesced 1-4 KiB segment of z and of w.  One Philox block per lane gives
// the lane's four noise values.  A 256-thread workgroup holds four rows of
// one 256-pair tile; grid = (row blocks of the colour) x (pair tiles of this
// launch).  The host may split a sweep into passes over groups of tiles so a
// tile's state stays cache-resident across the colours of the pass.
#include "device_common.h"
#include "sweep.h"

// Tuning knobs (compile time).
#ifndef MCINV_GATHER_U4
#define MCINV_GATHER_U4 2        // neighbours per gather chunk, 4-byte state
#endif
#ifndef MCINV_GATHER_U8
#define MCINV_GATHER_U8 2        // 8-byte state (fp64, complex64)
#endif
#ifndef MCINV_GATHER_U16
#define MCINV_GATHER_U16 1       // 16-byte state (complex128)
#endif
#ifndef MCINV_GATHER_HERM_U4
#define MCINV_GATHER_HERM_U4 4   // single-draw mode, 4-byte state: one load per neighbour, so twice the chunk
#endif

namespace mcinv {

template <typename V>
struct alignas(16) Quad {
    V v[4];
};

template <typename V>
__device__ inline Quad<V> load_quad(const V* p)
{
    return *reinterpret_cast<const Quad<V>*>(p);
}

// The new state row is read again only by rows of later colours.  When every
// launch covers all pair tiles those reads come in later launches, so the row
// is stored non-temporally and does not displace the neighbour slices the
// current launch is gathering (measured 3-5% faster); in tile passes the later
// colours of the same pass gather it soon after, and a temporal store keeps it
// in the caches for them.
template <typename V>
__device__ inline void store_quad(V* p, const Quad<V>& q, bool nt)
{
    static_assert(sizeof(Quad<V>) % 16 == 0, "quads are whole 16-byte vectors");
    const uint4* src = reinterpret_cast<const uint4*>(&q);
    uint4* dst = reinterpret_cast<uint4*>(p);
    if (nt) {
#pragma unroll
        for (int k = 0; k < (int)(sizeof(Quad<V>) / 16); ++k) {
            __builtin_nontemporal_store(src[k].x, &dst[k].x);
            __builtin_nontemporal_store(src[k].y, &dst[k].y);
            __builtin_nontemporal_store(src[k].z, &dst[k].z);
            __builtin_nontemporal_store(src[k].w, &dst[k].w);
        }
    } else {
#pragma unroll
        for (int k = 0; k < (int)(sizeof(Quad<V>) / 16); ++k) dst[k] = src[k];
    }
}

// product z * conj(w) in double
template <typename R>
__device__ inline void prod_acc(R z, R w, double& re, double&)
{
    re += (double)z * (double)w;
}
template <typename R>
__device__ inline void prod_acc(Cx<R> z, Cx<R> w, double& re, double& im)
{
    const double zr = z.re, zi = z.im, wr = w.re, wi = w.im;
    re += zr * wr + zi * wi;
    im += zi * wr - zr * wi;
}

// HERM: C is hermitian with a positive diagonal, so w = z at every step (the
// single-draw Gauss-Seidel sampler of eq 2): only z is gathered and stored,
// and the moments use z conj(z).
template <typename V, bool SAMPLE, bool HERM>
__global__ __launch_bounds__(256) void k_sweep(const SweepArgs<V> a)
{
    using R = typename Real<V>::type;
    constexpr bool CPLX = IsCx<V>::value;
    __shared__ double lds_tr[4][2];

    const int lane = threadIdx.x & (kWave - 1);
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    uint32_t bx = blockIdx.x, by = blockIdx.y;
    if (a.xcd_order == 3) {
        // pair tiles fastest: the tiles of one row block are dispatched one
        // after another, so the slices of a neighbour row are fetched
        // together (one contiguous run of the row's pairs) rather than one
        // tile at a time across the whole launch
        const uint32_t lin = blockIdx.x + gridDim.x * blockIdx.y;
        by = lin % gridDim.y;
        bx = lin / gridDim.y;
    } else if (a.xcd_order == 2) {
        // XCD x takes runs of 16 consecutive row blocks of a tile: workgroups
        // k, k + 8, ... (one XCD) sweep neighbouring rows, whose neighbour
        // slices then share that XCD's L2 (pays off on lattice-like patterns)
        constexpr uint32_t C = 16;
        const uint32_t k = blockIdx.x, whole = gridDim.x / (8 * C) * (8 * C);
        if (k < whole) {
            const uint32_t r = k % (8 * C);
            bx = k - r + (r % 8) * C + r / 8;
        }
    } else if (a.xcd_order == 1) {
        // XCD-aware order: workgroups are dealt round-robin to the 8 XCDs, so
        // give XCD x one contiguous range of (tile, row block) indices of this
        // launch (each XCD's L2 then holds the neighbour slices of its own
        // tiles; pays off on structured patterns, see the launch autotuner).
        const uint32_t total = gridDim.x * gridDim.y;
        const uint32_t lin = blockIdx.x + gridDim.x * blockIdx.y;
        const uint32_t xcd = lin % 8u, idx = lin / 8u, per = total / 8u, extra = total % 8u;
        const uint32_t remap = xcd * per + (xcd < extra ? xcd : extra) + idx;
        bx = remap % gridDim.x;
        by = remap / gridDim.x;
    }
    const int64_t tile = a.tile0 + by;
    const int64_t q = a.row_begin + (int64_t)bx * 4 + wid;
    const int64_t p0 = tile * kPairsPerWave + lane * kPairsPerLane;
    const bool row_ok = q < a.row_end;
    const bool active = p0 < a.ld;
    double tre = 0.0, tim = 0.0;

    if (row_ok) {
        const RowRec rr = a.rows[q];
        V az[4], aw[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) az[j] = aw[j] = vzero<V>();

        // Gather in chunks of U neighbours: all 2U state loads of a chunk are
        // issued before the first multiply (memory-level parallelism per wave).
        // A chunk's unused slots reload entry 0 with zero coefficients.
        constexpr int U = (HERM && sizeof(V) == 4)
                              ? MCINV_GATHER_HERM_U4
                              : (sizeof(V) >= 16 ? MCINV_GATHER_U16 : (sizeof(V) >= 8 ? MCINV_GATHER_U8 : MCINV_GATHER_U4));
        if (active) {
            const Entry<V>* e = a.ent + rr.begin;
            const int cnt = rr.count;
            for (int base = 0; base < cnt; base += U) {
                Quad<V> xs[U], ys[U];
                V us[U], vs[U];
#pragma unroll
                for (int t = 0; t < U; ++t) {
                    const bool ok = base + t < cnt;
                    const Entry<V> en = e[ok ? base + t : 0];
                    us[t] = ok ? en.u : vzero<V>();
                    vs[t] = ok ? en.v : vzero<V>();
                    const int64_t off = (int64_t)en.col * a.ld + p0;
                    xs[t] = load_quad(a.z + off);
                    if constexpr (!HERM) ys[t] = load_quad(a.w + off);
                }
#pragma unroll
                for (int t = 0; t < U; ++t)
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        az[j] = mul_add(us[t], xs[t].v[j], az[j]);
                        if constexpr (!HERM) aw[j] = mul_add(vs[t], ys[t].v[j], aw[j]);
                    }
            }
        }

        R phi[4];
        noise4<R>(a.key0, a.key1, rr.orig, a.sweep, a.pair_block0 + (uint32_t)(p0 >> 2), a.stream, a.noise, phi);
        const Scales<V> s = a.sc[q];
        Quad<V> zn, wn;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            zn.v[j] = noisy_update(s.a, phi[j], az[j]);
            wn.v[j] = HERM ? zn.v[j] : noisy_update(s.b, phi[j], aw[j]);
        }
        if (active) {
            store_quad(a.z + q * a.ld + p0, zn, a.nt_stores != 0);
            if constexpr (!HERM) store_quad(a.w + q * a.ld + p0, wn, a.nt_stores != 0);
        }

        // Divergence guard (Sec. 2.2): a runaway or non-finite state.
        R mag = R(0);
#pragma unroll
        for (int j = 0; j < 4; ++j) mag = fmax(mag, fmax(magnitude(zn.v[j]), magnitude(wn.v[j])));
        const bool bad = active && !(mag < a.thresh);
        if (__any(bad) && lane == 0) atomicOr(a.flag, 1);

        if constexpr (SAMPLE) {
            if (active) {
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    if (p0 + j < a.P) prod_acc(zn.v[j], wn.v[j], tre, tim);
            }
            const int lg = 1 << a.lg_shift;
            for (int off = 1; off < lg; off <<= 1) {
                tre += __shfl_xor(tre, off);
                if constexpr (CPLX) tim += __shfl_xor(tim, off);
            }
            if (a.diag != nullptr && active && (lane & (lg - 1)) == 0) {
                const int cpt = kWave >> a.lg_shift;
                const int64_t at = (tile * a.n + q) * cpt + (lane >> a.lg_shift);
                if constexpr (CPLX) {
                    double* d = a.diag + 2 * at;
                    d[0] += tre;
                    d[1] += tim;
                } else {
                    a.diag[at] += tre;
                }
            }
            for (int off = lg; off < kWave; off <<= 1) {
                tre += __shfl_xor(tre, off);
                if constexpr (CPLX) tim += __shfl_xor(tim, off);
            }
        }
    }

    if constexpr (SAMPLE) {
        if (a.tpart != nullptr) {
            if (lane == 0) {
                lds_tr[wid][0] = row_ok ? tre : 0.0;
                lds_tr[wid][1] = row_ok ? tim : 0.0;
            }
            __syncthreads();
            if (threadIdx.x == 0) {
                const int64_t slot = tile * gridDim.x + bx;
                const double r = ((lds_tr[0][0] + lds_tr[1][0]) + lds_tr[2][0]) + lds_tr[3][0];
                if constexpr (CPLX) {
                    const double i = ((lds_tr[0][1] + lds_tr[1][1]) + lds_tr[2][1]) + lds_tr[3][1];
                    a.tpart[2 * slot] = r;
                    a.tpart[2 * slot + 1] = i;
                } else {
                    a.tpart[slot] = r;
                }
            }
        }
    }
}

template <typename V>
hipError_t launch_sweep(const SweepArgs<V>& a, int64_t ntiles, bool sample, bool herm, hipStream_t stream)
{
    const int64_t rows = a.row_end - a.row_begin;
    if (rows <= 0 || ntiles <= 0) return hipSuccess;
    const dim3 grid((unsigned)((rows + 3) / 4), (unsigned)ntiles);
    if (herm) {
        if (sample)
            k_sweep<V, true, true><<<grid, dim3(256), 0, stream>>>(a);
        else
            k_sweep<V, false, true><<<grid, dim3(256), 0, stream>>>(a);
    } else {
        if (sample)
            k_sweep<V, true, false><<<grid, dim3(256), 0, stream>>>(a);
        else
            k_sweep<V, false, false><<<grid, dim3(256), 0, stream>>>(a);
    }
    return hipGetLastError();
}

template hipError_t launch_sweep<float>(const SweepArgs<float>&, int64_t, bool, bool, hipStream_t);
template hipError_t launch_sweep<double>(const SweepArgs<double>&, int64_t, bool, bool, hipStream_t);
template hipError_t launch_sweep<Cx<float>>(const SweepArgs<Cx<float>>&, int64_t, bool, bool, hipStream_t);
template hipError_t launch_sweep<Cx<double>>(const SweepArgs<Cx<double>>&, int64_t, bool, bool, hipStream_t);

// --------------------------------------------------------------------------
// Noise values for given (row, sweep, pair) triples, as the sweep draws them.
template <typename R>
__global__ __launch_bounds__(256) void k_noise_values(uint32_t k0, uint32_t k1, uint32_t stream,
                                                      int32_t kind, int64_t count, const int64_t* row,
                                                      const int64_t* sweep, const int64_t* pair,
                                                      double* out)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= count) return;
    R v[4];
    noise4<R>(k0, k1, (uint32_t)row[t], (uint32_t)sweep[t], (uint32_t)(pair[t] >> 2), stream, kind, v);
    out[t] = (double)v[pair[t] & 3];
}

hipError_t launch_noise_values(bool fp64, uint64_t seed, uint32_t stream_id, int32_t kind, int64_t count,
                               const int64_t* row, const int64_t* sweep, const int64_t* pair, double* out,
                               hipStream_t stream)
{
    if (count <= 0) return hipSuccess;
    const uint32_t k0 = (uint32_t)(seed & 0xffffffffu), k1 = (uint32_t)(seed >> 32);
    const unsigned blocks = (unsigned)((count + 255) / 256);
    if (fp64)
        k_noise_values<double><<<dim3(blocks), dim3(256), 0, stream>>>(k0, k1, stream_id, kind, count, row, sweep, pair, out);
    else
        k_noise_values<float><<<dim3(blocks), dim3(256), 0, stream>>>(k0, k1, stream_id, kind, count, row, sweep, pair, out);
    return hipGetLastError();
}

}  // namespace mcinv
