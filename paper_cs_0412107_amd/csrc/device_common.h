// Device-side building blocks shared by the mcinv kernels (gfx950, wave64).
//
// Noise (Sec. 2, eqs 5a/5b: zero mean, identity covariance, independent per
// sweep): Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) keyed by the seed
// with counter (row, sweep, pair/4, stream); the four 32-bit outputs become
// four N(0,1) values by the Box-Muller transform (Box & Muller, 1958) on
// u = ((x >> 9) + 1/2) 2^-23, or Z2 values (sign bit), or zeros.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mcinv {

constexpr int kWave = 64;           // CDNA wavefront width
constexpr int kPairsPerLane = 4;    // one Philox block per lane
constexpr int kPairsPerWave = kWave * kPairsPerLane;

enum NoiseKind : int32_t { kNoiseNormal = 0, kNoiseRademacher = 1, kNoiseNone = 2 };

// ---------------------------------------------------------------- complex --
template <typename R>
struct alignas(2 * sizeof(R)) Cx {
    R re, im;
};

template <typename R> struct Real { using type = R; };
template <typename R> struct Real<Cx<R>> { using type = R; };

template <typename V> struct IsCx { static constexpr bool value = false; };
template <typename R> struct IsCx<Cx<R>> { static constexpr bool value = true; };

template <typename R> __host__ __device__ inline R zero_of(R*) { return R(0); }
template <typename R> __host__ __device__ inline Cx<R> zero_of(Cx<R>*) { return Cx<R>{R(0), R(0)}; }
template <typename V> __host__ __device__ inline V vzero() { return zero_of((V*)nullptr); }

template <typename R> __device__ inline bool is_zero(R x) { return x == R(0); }
template <typename R> __device__ inline bool is_zero(Cx<R> x) { return x.re == R(0) && x.im == R(0); }

// acc + u * x
template <typename R> __device__ inline R mul_add(R u, R x, R acc) { return __builtin_fma(u, x, acc); }
__device__ inline float mul_add(float u, float x, float acc) { return __builtin_fmaf(u, x, acc); }
template <typename R> __device__ inline Cx<R> mul_add(Cx<R> u, Cx<R> x, Cx<R> acc)
{
    acc.re = mul_add(u.re, x.re, acc.re);
    acc.re = mul_add(-u.im, x.im, acc.re);
    acc.im = mul_add(u.re, x.im, acc.im);
    acc.im = mul_add(u.im, x.re, acc.im);
    return acc;
}

// a * phi - s   (phi real)
template <typename R> __device__ inline R noisy_update(R a, R phi, R s) { return a * phi - s; }
template <typename R> __device__ inline Cx<R> noisy_update(Cx<R> a, R phi, Cx<R> s)
{
    return Cx<R>{a.re * phi - s.re, a.im * phi - s.im};
}

template <typename R> __device__ inline R magnitude(R x) { return x < R(0) ? -x : x; }
template <typename R> __device__ inline R magnitude(Cx<R> x) { return fmax(magnitude(x.re), magnitude(x.im)); }

// ----------------------------------------------------------------- Philox --
struct Philox {
    static constexpr uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    static constexpr uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;

    __device__ static inline void block(uint32_t& c0, uint32_t& c1, uint32_t& c2, uint32_t& c3,
                                        uint32_t k0, uint32_t k1)
    {
#pragma unroll
        for (int r = 0; r < 10; ++r) {
            // one 32 x 32 -> 64-bit multiply gives both halves
            const uint64_t p0 = (uint64_t)M0 * c0;
            const uint64_t p1 = (uint64_t)M1 * c2;
            const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
            const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
            c0 = n0;
            c1 = (uint32_t)p1;
            c2 = n2;
            c3 = (uint32_t)p0;
            k0 += W0;
            k1 += W1;
        }
    }
};

template <typename R> __device__ inline R uniform_open(uint32_t x);
template <> __device__ inline float uniform_open<float>(uint32_t x)
{
    return ((float)(x >> 9) + 0.5f) * 0x1p-23f;
}
template <> __device__ inline double uniform_open<double>(uint32_t x)
{
    return ((double)(x >> 9) + 0.5) * 0x1p-23;
}

// fp32 sin/cos of 2 pi u on the hardware units (argument in turns): on the 2^23
// possible u the absolute error is 1.3e-7 (measured against fp64), below the
// fp32 state's own rounding, and the range reduction of sincospif is avoided.
#ifndef MCINV_FAST_SINCOS
#define MCINV_FAST_SINCOS 1
#endif

template <typename R> __device__ inline void sincos_2pi(R u, R* s, R* c);
template <> __device__ inline void sincos_2pi<float>(float u, float* s, float* c)
{
#if MCINV_FAST_SINCOS
    *s = __builtin_amdgcn_sinf(u);
    *c = __builtin_amdgcn_cosf(u);
#else
    sincospif(2.0f * u, s, c);
#endif
}
template <> __device__ inline void sincos_2pi<double>(double u, double* s, double* c) { sincospi(2.0 * u, s, c); }

// The four noise values of pairs 4*quad .. 4*quad+3 at (row, sweep).
template <typename R>
__device__ inline void noise4(uint32_t k0, uint32_t k1, uint32_t row, uint32_t sweep, uint32_t quad,
                              uint32_t stream, int32_t kind, R out[4])
{
    uint32_t c0 = row, c1 = sweep, c2 = quad, c3 = stream;
    Philox::block(c0, c1, c2, c3, k0, k1);
    if (kind == kNoiseNormal) {
        const R u0 = uniform_open<R>(c0), u1 = uniform_open<R>(c1);
        const R u2 = uniform_open<R>(c2), u3 = uniform_open<R>(c3);
        const R r0 = sqrt(R(-2) * log(u0));
        const R r1 = sqrt(R(-2) * log(u2));
        R s0, co0, s1, co1;
        sincos_2pi<R>(u1, &s0, &co0);
        sincos_2pi<R>(u3, &s1, &co1);
        out[0] = r0 * co0;
        out[1] = r0 * s0;
        out[2] = r1 * co1;
        out[3] = r1 * s1;
    } else if (kind == kNoiseRademacher) {
        out[0] = (c0 >> 31) ? R(-1) : R(1);
        out[1] = (c1 >> 31) ? R(-1) : R(1);
        out[2] = (c2 >> 31) ? R(-1) : R(1);
        out[3] = (c3 >> 31) ? R(-1) : R(1);
    } else {
        out[0] = out[1] = out[2] = out[3] = R(0);
    }
}

// ----------------------------------------------------------- data layout --
// One sweep position (a row of the permuted matrix).
struct RowRec {
    int64_t begin;   // first merged off-diagonal entry
    int32_t count;   // number of merged off-diagonal entries
    uint32_t orig;   // original row index (Philox counter word 0)
};

// One off-diagonal entry of the merged symmetric pattern at position q:
//   u = c_ij / c_ii           (z update, eq 4; 0 if c_ij is not stored)
//   v = conj(c_ji) / conj(c_ii) (w update, eq 5; 0 if c_ji is not stored)
template <typename V>
struct Entry {
    int32_t col;     // position of the neighbour row j
    int32_t pad;
    V u;
    V v;
};

// Noise scales of one position: a (z) and b (w), a conj(b) = 1/c_ii.
template <typename V>
struct Scales {
    V a;
    V b;
};

}  // namespace mcinv
