// Device-side building blocks of libkpm (gfx950): 16-byte vector types,
// division by run-time constants, the Philox4x64-10 generator, double-double
// accumulation and wave/block reductions.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace kpm {

// ---------------------------------------------------------------------------
// 16-byte vector of scalars: every thread moves one such chunk per stream.
// ---------------------------------------------------------------------------
template <typename S> struct V16;
template <> struct V16<float> {
    typedef float T __attribute__((ext_vector_type(4)));
    enum { W = 4 };
};
template <> struct V16<double> {
    typedef double T __attribute__((ext_vector_type(2)));
    enum { W = 2 };
};

template <typename S>
__device__ __forceinline__ typename V16<S>::T ld16(const S *p)
{
    return *reinterpret_cast<const typename V16<S>::T *>(p);
}
template <typename S>
__device__ __forceinline__ typename V16<S>::T ld16_stream(const S *p)
{
    return __builtin_nontemporal_load(reinterpret_cast<const typename V16<S>::T *>(p));
}
template <typename S>
__device__ __forceinline__ void st16_stream(S *p, typename V16<S>::T v)
{
    __builtin_nontemporal_store(v, reinterpret_cast<typename V16<S>::T *>(p));
}

// ---------------------------------------------------------------------------
// Unsigned 32-bit division by a run-time constant d >= 1 (Granlund and
// Montgomery, "Division by invariant integers using multiplication", PLDI'94):
// with s = ceil(log2 d) and m = floor(2^32 (2^s - d) / d) + 1,
// floor(n / d) = (mulhi(m, n) + n) >> s for every 32-bit n.
// ---------------------------------------------------------------------------
struct FastDiv {
    uint32_t d, m, s, pad;
};

__host__ __device__ __forceinline__ uint32_t fdiv(uint32_t n, FastDiv f)
{
    uint32_t hi = (uint32_t)(((uint64_t)f.m * (uint64_t)n) >> 32);
    return (uint32_t)(((uint64_t)hi + (uint64_t)n) >> f.s);
}

static inline FastDiv make_fastdiv(uint32_t d)
{
    FastDiv f;
    f.d = d;
    uint32_t s = 0;
    while ((uint64_t(1) << s) < (uint64_t)d) ++s;
    f.s = s;
    f.m = (uint32_t)((((uint64_t(1) << 32) * ((uint64_t(1) << s) - (uint64_t)d)) / (uint64_t)d) + 1);
    f.pad = 0;
    return f;
}

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
// as 1, 2, 3", SC'11): ten rounds of two 64x64->128 multiplications with the
// round multipliers, the key bumped by the Weyl constants between rounds.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void philox4x64_10(uint64_t &c0, uint64_t &c1, uint64_t &c2, uint64_t &c3,
                                              uint64_t k0, uint64_t k1)
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        uint64_t hi0 = __umul64hi(M0, c0), lo0 = M0 * c0;
        uint64_t hi1 = __umul64hi(M1, c2), lo1 = M1 * c2;
        uint64_t n0 = hi1 ^ c1 ^ k0;
        uint64_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += W0;
        k1 += W1;
    }
}

// ---------------------------------------------------------------------------
// double-double arithmetic (error-free transformations: Knuth's two-sum,
// the fma two-product; accumulation as in Ogita, Rump, Oishi, "Accurate sum
// and dot product", SIAM J. Sci. Comput. 26, 2005).
// ---------------------------------------------------------------------------
struct dd {
    double hi, lo;
};

__device__ __forceinline__ dd dd_two_sum(double a, double b)
{
    double s = a + b;
    double v = s - a;
    double e = (a - (s - v)) + (b - v);
    return dd{s, e};
}
__device__ __forceinline__ dd dd_fast_two_sum(double a, double b)
{
    double s = a + b;
    double e = b - (s - a);
    return dd{s, e};
}
__device__ __forceinline__ dd dd_add(dd x, dd y)
{
    dd s = dd_two_sum(x.hi, y.hi);
    dd t = dd_two_sum(x.lo, y.lo);
    s.lo += t.hi;
    s = dd_fast_two_sum(s.hi, s.lo);
    s.lo += t.lo;
    return dd_fast_two_sum(s.hi, s.lo);
}
// (s, c) += x*y exactly up to the error term c, which is summed in FP64.
__device__ __forceinline__ void dot2_acc(double &s, double &c, double x, double y)
{
    double p = x * y;
    double pe = fma(x, y, -p);
    double t = s + p;
    double v = t - s;
    double e = (s - (t - v)) + (p - v);
    s = t;
    c += e + pe;
}
__device__ __forceinline__ dd dd_div_d(dd x, double b)
{
    double q1 = x.hi / b;
    double p = q1 * b;
    double pe = fma(q1, b, -p);
    double r = ((x.hi - p) - pe) + x.lo;
    double q2 = r / b;
    return dd_fast_two_sum(q1, q2);
}

__device__ __forceinline__ double shfl_xor_d(double v, int mask)
{
    return __shfl_xor(v, mask, 64);
}

}  // namespace kpm
