// Kernels of libkpm for gfx950.
//
// The hot path is the fused recursion step (Eq. (rn) of Zhang et al. 2011):
//     r_{n+1} = 2 H~ r_n - r_{n-1},  written over r_{n-1},
// with the two dot products <r_{n+1}|r_{n+1}> and Re<r_{n+1}|r_n> that the
// doubling identities turn into mu_{2n+2} and mu_{2n+1}, taken from registers
// in the same pass.  Vectors are stored site-major: the R vectors (or 2R
// interleaved re/im scalars) of site i are contiguous, padded to 16 bytes, so
// one thread moves one 16-byte chunk of one site per stream and a wavefront
// reads whole cache lines; the neighbours of a site are the same chunk of the
// neighbouring sites.
//
// Work is cut into tiles of 256*TPT chunks.  Each tile leaves one reduction
// partial (FP64 sums of its dot products) in a ring of per-step slots; a
// separate kernel later sums the partials of a step over the tiles in a fixed
// order.  Results therefore do not depend on the launch grid or on which other
// instances share the launch.  The blocks of one instance walk its tiles in a
// band per XCD: block b (b mod 8 = its XCD under round-robin dispatch) covers
// tiles of the b-th eighth of the instance, so neighbouring rows/planes are
// read by blocks of the same XCD and hit its L2.
#pragma once

#include "kpm_device.hpp"

namespace kpm {

enum OpKind { OP_REAL2 = 0, OP_REAL3 = 1, OP_SPIN2 = 2, OP_SPIN3 = 3, OP_CSR_R = 4, OP_CSR_C = 5, OP_COUNT = 6 };
enum { VEC_RADEMACHER = 0, VEC_PHASE = 1, VEC_UNIT = 2 };
constexpr int BLOCK = 256;

// One solve inside a launch (device-resident table entry).
struct Inst {
    int32_t opk;
    int32_t has_diag;
    uint32_t Lx, Ly, Lz, N;
    FastDiv fLx, fLy, fC;
    uint32_t C;        // 16-byte chunks per site
    uint32_t Rs;       // scalars per site (C * W)
    uint32_t nel;      // N * C
    uint32_t tiles;    // ceil(nel / (256 * TPT))
    uint32_t nb;       // blocks given to this instance (multiple of 8)
    uint32_t block0;   // first block of this instance in the grid (multiple of 8)
    int32_t tpt;
    int32_t cplx;      // data stored as interleaved complex
    int32_t M, K, R, vec;
    int32_t step0;     // recursion step n = step0 + (launch offset k)
    int32_t pslots;    // ring slots of partials
    uint64_t seed, instance;
    double norm;       // N R (random kinds) or R (unit vectors)
    const void *diag;  // S[N]
    const void *bond;  // S[N][dim][2]: H~_{i, i+e_ax}
    const void *hop;   // S[1]: H~_ij of the real lattice
    const int64_t *row_ptr;
    const int32_t *col;
    const void *val;   // S[nnz] or S[nnz][2]
    void *buf0, *buf1;
    double *partial;   // [pslots][tiles][4]
    double *dots;      // [K+1][4] = (nn.hi, nn.lo, nm.hi, nm.lo)
    double *mu;        // [M]
};

// ---------------------------------------------------------------------------
// arithmetic policies
// FP64 follows the oracle's order with no fused operations (the library is
// compiled with -ffp-contract=off), so the FP64 vectors are bitwise equal to
// a plain sequential evaluation.  FP32 uses fma freely.
// ---------------------------------------------------------------------------
template <typename S> struct Arith;
template <> struct Arith<double> {
    typedef V16<double>::T T;
    static __device__ __forceinline__ T mac(T acc, double h, T v) { return acc + h * v; }
    static __device__ __forceinline__ void cmul(double &ar, double &ai, double hr, double hi, double vr, double vi)
    {
        ar = hr * vr - hi * vi;
        ai = hr * vi + hi * vr;
    }
    static __device__ __forceinline__ void cmac(double &ar, double &ai, double hr, double hi, double vr, double vi)
    {
        ar = ar + (hr * vr - hi * vi);
        ai = ai + (hr * vi + hi * vr);
    }
};
template <> struct Arith<float> {
    typedef V16<float>::T T;
    static __device__ __forceinline__ T mac(T acc, float h, T v)
    {
        T hv = h;
        return __builtin_elementwise_fma(hv, v, acc);
    }
    static __device__ __forceinline__ void cmul(float &ar, float &ai, float hr, float hi, float vr, float vi)
    {
        ar = fmaf(hr, vr, -hi * vi);
        ai = fmaf(hr, vi, hi * vr);
    }
    static __device__ __forceinline__ void cmac(float &ar, float &ai, float hr, float hi, float vr, float vi)
    {
        ar = fmaf(hr, vr, fmaf(-hi, vi, ar));
        ai = fmaf(hr, vi, fmaf(hi, vr, ai));
    }
};

// Dot-product accumulators: (sum, error) pairs in FP64 for FP64 vectors; for
// FP32 vectors the products are exact in FP64 and a plain FP64 sum suffices.
template <typename S> struct Dots;
template <> struct Dots<double> {
    double s0 = 0.0, c0 = 0.0, s1 = 0.0, c1 = 0.0;
    __device__ __forceinline__ void add(V16<double>::T o, V16<double>::T v)
    {
#pragma unroll
        for (int l = 0; l < 2; ++l) {
            dot2_acc(s0, c0, o[l], o[l]);
            dot2_acc(s1, c1, o[l], v[l]);
        }
    }
    __device__ __forceinline__ void norm_only(V16<double>::T o)
    {
#pragma unroll
        for (int l = 0; l < 2; ++l) dot2_acc(s0, c0, o[l], o[l]);
    }
    static constexpr bool DD = true;
};
template <> struct Dots<float> {
    double s0 = 0.0, c0 = 0.0, s1 = 0.0, c1 = 0.0;
    __device__ __forceinline__ void add(V16<float>::T o, V16<float>::T v)
    {
#pragma unroll
        for (int l = 0; l < 4; ++l) {
            double a = (double)o[l];
            s0 = fma(a, a, s0);
            s1 = fma(a, (double)v[l], s1);
        }
    }
    __device__ __forceinline__ void norm_only(V16<float>::T o)
    {
#pragma unroll
        for (int l = 0; l < 4; ++l) {
            double a = (double)o[l];
            s0 = fma(a, a, s0);
        }
    }
    static constexpr bool DD = false;
};

// Sum (x0 + x1, x2 + x3) over the block in a fixed order; thread 0 stores
// the four doubles (hi, lo, hi, lo) at dst.
template <bool DD>
__device__ __forceinline__ void block_reduce_store(double x0, double x1, double x2, double x3, double *dst)
{
    __shared__ double red[BLOCK / 64][4];
    if (DD) {
        dd a = dd_fast_two_sum(x0, x1), b = dd_fast_two_sum(x2, x3);
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            dd oa{shfl_xor_d(a.hi, off), shfl_xor_d(a.lo, off)};
            dd ob{shfl_xor_d(b.hi, off), shfl_xor_d(b.lo, off)};
            a = dd_add(a, oa);
            b = dd_add(b, ob);
        }
        x0 = a.hi; x1 = a.lo; x2 = b.hi; x3 = b.lo;
    } else {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            x0 += shfl_xor_d(x0, off);
            x2 += shfl_xor_d(x2, off);
        }
        x1 = 0.0;
        x3 = 0.0;
    }
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) {
        red[w][0] = x0; red[w][1] = x1; red[w][2] = x2; red[w][3] = x3;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        dd a{red[0][0], red[0][1]}, b{red[0][2], red[0][3]};
#pragma unroll
        for (int k = 1; k < BLOCK / 64; ++k) {
            if (DD) {
                a = dd_add(a, dd{red[k][0], red[k][1]});
                b = dd_add(b, dd{red[k][2], red[k][3]});
            } else {
                a.hi += red[k][0];
                b.hi += red[k][2];
            }
        }
        dst[0] = a.hi; dst[1] = a.lo; dst[2] = b.hi; dst[3] = b.lo;
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// start vectors
// ---------------------------------------------------------------------------
// The four Philox words for site i and vectors 4*rq .. 4*rq+3.
__device__ __forceinline__ void start_words(uint64_t seed, uint64_t instance, uint32_t i, uint32_t rq, uint64_t w[4])
{
    uint64_t c0 = i, c1 = rq, c2 = instance, c3 = 0;
    philox4x64_10(c0, c1, c2, c3, seed, 4);
    w[0] = c0; w[1] = c1; w[2] = c2; w[3] = c3;
}
// (re, im) of xi_{r,i} given its Philox word.
__device__ __forceinline__ void start_value(int vec, uint64_t word, uint64_t instance, uint32_t N, uint32_t i,
                                            uint32_t r, double &re, double &im)
{
    if (vec == VEC_RADEMACHER) {
        re = (word >> 63) ? -1.0 : 1.0;
        im = 0.0;
    } else if (vec == VEC_PHASE) {
        double u = (double)(word >> 11) * 0x1p-53;
        double phi = 6.283185307179586 * u;
        sincos(phi, &im, &re);
    } else {
        uint64_t j = (instance + (uint64_t)r) % (uint64_t)N;
        re = (j == (uint64_t)i) ? 1.0 : 0.0;
        im = 0.0;
    }
}

template <typename S, int TPT>
__global__ __launch_bounds__(BLOCK) void k_init(const Inst *__restrict__ tab, const uint32_t *__restrict__ map8)
{
    typedef typename V16<S>::T T;
    constexpr int W = V16<S>::W;
    const uint32_t h = map8 ? map8[blockIdx.x >> 3] : 0u;
    const Inst *I = tab + h;
    if (I->step0 != 0) return;
    const uint32_t bl = blockIdx.x - I->block0;
    const uint32_t x8 = bl & 7u, j = bl >> 3, q = I->nb >> 3;
    const uint32_t tiles = I->tiles;
    const uint32_t tb = (uint32_t)(((uint64_t)tiles * x8) >> 3);
    const uint32_t te = (uint32_t)(((uint64_t)tiles * (x8 + 1)) >> 3);
    S *out = (S *)I->buf0;
    double *part = I->partial;     // slot 0
    for (uint32_t t = tb + j; t < te; t += q) {
        Dots<S> acc;
#pragma unroll
        for (int u = 0; u < TPT; ++u) {
            const uint32_t e = t * (uint32_t)(BLOCK * TPT) + (uint32_t)(u * BLOCK) + threadIdx.x;
            if (e < I->nel) {
                const uint32_t i = fdiv(e, I->fC);
                const uint32_t c = e - i * I->C;
                const uint32_t k0 = c * W;                    // first scalar of the chunk
                const uint32_t r0 = I->cplx ? k0 / 2 : k0;    // first vector of the chunk
                uint64_t w[4] = {0, 0, 0, 0};
                if (I->vec != VEC_UNIT) start_words(I->seed, I->instance, i, r0 / 4, w);
                T v;
                if (I->cplx) {
#pragma unroll
                    for (int l = 0; l < W / 2; ++l) {
                        const uint32_t r = r0 + l;
                        double re = 0.0, im = 0.0;
                        if (r < (uint32_t)I->R) start_value(I->vec, w[r & 3], I->instance, I->N, i, r, re, im);
                        v[2 * l] = (S)re;
                        v[2 * l + 1] = (S)im;
                    }
                } else {
#pragma unroll
                    for (int l = 0; l < W; ++l) {
                        const uint32_t r = r0 + l;
                        double re = 0.0, im = 0.0;
                        if (r < (uint32_t)I->R) start_value(I->vec, w[r & 3], I->instance, I->N, i, r, re, im);
                        v[l] = (S)re;
                    }
                }
                *reinterpret_cast<T *>(out + (size_t)i * I->Rs + k0) = v;
                acc.norm_only(v);
            }
        }
        block_reduce_store<Dots<S>::DD>(acc.s0, acc.c0, acc.s1, acc.c1, part + (size_t)t * 4);
    }
}

// ---------------------------------------------------------------------------
// the fused recursion step
// ---------------------------------------------------------------------------
template <typename S, int OPK>
__device__ __forceinline__ void step_elem(const Inst *__restrict__ I, uint32_t e, const S *__restrict__ cur,
                                          S *__restrict__ nxt, bool first, Dots<S> &acc)
{
    typedef typename V16<S>::T T;
    typedef Arith<S> A;
    constexpr int W = V16<S>::W;
    const uint32_t i = fdiv(e, I->fC);
    const uint32_t c = e - i * I->C;
    const uint32_t Rs = I->Rs;
    const size_t cw = (size_t)c * W;
    const size_t off = (size_t)i * Rs + cw;
    const T v = ld16(cur + off);
    T out;
    if constexpr (OPK <= OP_SPIN3) {
        constexpr bool D3 = (OPK == OP_REAL3 || OPK == OP_SPIN3);
        constexpr bool SPIN = (OPK == OP_SPIN2 || OPK == OP_SPIN3);
        const uint32_t Lx = I->Lx, Ly = I->Ly;
        const uint32_t yq = fdiv(i, I->fLx);
        const uint32_t x = i - yq * Lx;
        uint32_t y = yq, z = 0;
        if (D3) {
            z = fdiv(yq, I->fLy);
            y = yq - z * Ly;
        }
        const uint32_t xm = (x == 0) ? i + (Lx - 1) : i - 1;
        const uint32_t xp = (x == Lx - 1) ? i - (Lx - 1) : i + 1;
        const uint32_t ym = (y == 0) ? i + (Ly - 1) * Lx : i - Lx;
        const uint32_t yp = (y == Ly - 1) ? i - (Ly - 1) * Lx : i + Lx;
        uint32_t zm = 0, zp = 0;
        if (D3) {
            const uint32_t Pz = Lx * Ly, Lz = I->Lz;
            zm = (z == 0) ? i + (Lz - 1) * Pz : i - Pz;
            zp = (z == Lz - 1) ? i - (Lz - 1) * Pz : i + Pz;
        }
        const T vxm = ld16(cur + (size_t)xm * Rs + cw);
        const T vxp = ld16(cur + (size_t)xp * Rs + cw);
        const T vym = ld16(cur + (size_t)ym * Rs + cw);
        const T vyp = ld16(cur + (size_t)yp * Rs + cw);
        T vzm, vzp;
        if (D3) {
            vzm = ld16(cur + (size_t)zm * Rs + cw);
            vzp = ld16(cur + (size_t)zp * Rs + cw);
        }
        if constexpr (!SPIN) {
            const S hh = *(const S *)I->hop;
            T a;
            if (I->has_diag) {
                const S d = ((const S *)I->diag)[i];
                a = d * v;
                a = A::mac(a, hh, vxm);
            } else {
                a = hh * vxm;
            }
            a = A::mac(a, hh, vxp);
            a = A::mac(a, hh, vym);
            a = A::mac(a, hh, vyp);
            if (D3) {
                a = A::mac(a, hh, vzm);
                a = A::mac(a, hh, vzp);
            }
            out = a;
        } else {
            constexpr int DIM = D3 ? 3 : 2;
            const S *B = (const S *)I->bond;
            // slot order -x, +x, -y, +y[, -z, +z]; H~_{i,i-e} = conj(H~_{i-e,i})
            const S bxm_r = B[((size_t)xm * DIM + 0) * 2], bxm_i = -B[((size_t)xm * DIM + 0) * 2 + 1];
            const S bxp_r = B[((size_t)i * DIM + 0) * 2], bxp_i = B[((size_t)i * DIM + 0) * 2 + 1];
            const S bym_r = B[((size_t)ym * DIM + 1) * 2], bym_i = -B[((size_t)ym * DIM + 1) * 2 + 1];
            const S byp_r = B[((size_t)i * DIM + 1) * 2], byp_i = B[((size_t)i * DIM + 1) * 2 + 1];
            S bzm_r = 0, bzm_i = 0, bzp_r = 0, bzp_i = 0;
            if (D3) {
                bzm_r = B[((size_t)zm * DIM + 2) * 2];
                bzm_i = -B[((size_t)zm * DIM + 2) * 2 + 1];
                bzp_r = B[((size_t)i * DIM + 2) * 2];
                bzp_i = B[((size_t)i * DIM + 2) * 2 + 1];
            }
            const bool hd = I->has_diag;
            const S d = hd ? ((const S *)I->diag)[i] : (S)0;
#pragma unroll
            for (int l = 0; l < W / 2; ++l) {
                S ar, ai;
                if (hd) {
                    ar = d * v[2 * l];
                    ai = d * v[2 * l + 1];
                    A::cmac(ar, ai, bxm_r, bxm_i, vxm[2 * l], vxm[2 * l + 1]);
                } else {
                    A::cmul(ar, ai, bxm_r, bxm_i, vxm[2 * l], vxm[2 * l + 1]);
                }
                A::cmac(ar, ai, bxp_r, bxp_i, vxp[2 * l], vxp[2 * l + 1]);
                A::cmac(ar, ai, bym_r, bym_i, vym[2 * l], vym[2 * l + 1]);
                A::cmac(ar, ai, byp_r, byp_i, vyp[2 * l], vyp[2 * l + 1]);
                if (D3) {
                    A::cmac(ar, ai, bzm_r, bzm_i, vzm[2 * l], vzm[2 * l + 1]);
                    A::cmac(ar, ai, bzp_r, bzp_i, vzp[2 * l], vzp[2 * l + 1]);
                }
                out[2 * l] = ar;
                out[2 * l + 1] = ai;
            }
        }
    } else {
        // CSR: the diagonal d_i first, then the off-diagonal entries in stored order
        const int64_t kb = I->row_ptr[i], ke = I->row_ptr[i + 1];
        const S d = ((const S *)I->diag)[i];
        if constexpr (OPK == OP_CSR_R) {
            T a = d * v;
            const S *val = (const S *)I->val;
            for (int64_t k = kb; k < ke; ++k) {
                const uint32_t jj = (uint32_t)I->col[k];
                if (jj == i) continue;
                a = A::mac(a, val[k], ld16(cur + (size_t)jj * Rs + cw));
            }
            out = a;
        } else {
            T a;
#pragma unroll
            for (int l = 0; l < W; ++l) a[l] = d * v[l];
            const S *val = (const S *)I->val;
            for (int64_t k = kb; k < ke; ++k) {
                const uint32_t jj = (uint32_t)I->col[k];
                if (jj == i) continue;
                const S hr = val[2 * k], hi = val[2 * k + 1];
                const T vj = ld16(cur + (size_t)jj * Rs + cw);
#pragma unroll
                for (int l = 0; l < W / 2; ++l) {
                    S ar = a[2 * l], ai = a[2 * l + 1];
                    A::cmac(ar, ai, hr, hi, vj[2 * l], vj[2 * l + 1]);
                    a[2 * l] = ar;
                    a[2 * l + 1] = ai;
                }
            }
            out = a;
        }
    }
    if (!first) {
        const T p = ld16_stream(nxt + off);
        out = (S)2 * out - p;
    }
    st16_stream(nxt + off, out);
    acc.add(out, v);
}

template <typename S, int OPK, int TPT>
__global__ __launch_bounds__(BLOCK) void k_step(const Inst *__restrict__ tab, const uint32_t *__restrict__ map8,
                                                int32_t k)
{
    const uint32_t h = map8 ? map8[blockIdx.x >> 3] : 0u;
    const Inst *I = tab + h;
    const int32_t n = I->step0 + k;
    if (n < 0 || n >= I->K) return;
    const uint32_t bl = blockIdx.x - I->block0;
    const uint32_t x8 = bl & 7u, j = bl >> 3, q = I->nb >> 3;
    const uint32_t tiles = I->tiles;
    const uint32_t tb = (uint32_t)(((uint64_t)tiles * x8) >> 3);
    const uint32_t te = (uint32_t)(((uint64_t)tiles * (x8 + 1)) >> 3);
    const S *cur = (const S *)((n & 1) ? I->buf1 : I->buf0);
    S *nxt = (S *)((n & 1) ? I->buf0 : I->buf1);
    const bool first = (n == 0);
    double *part = I->partial + (size_t)((n + 1) % I->pslots) * tiles * 4;
    for (uint32_t t = tb + j; t < te; t += q) {
        Dots<S> acc;
#pragma unroll
        for (int u = 0; u < TPT; ++u) {
            const uint32_t e = t * (uint32_t)(BLOCK * TPT) + (uint32_t)(u * BLOCK) + threadIdx.x;
            if (e < I->nel) step_elem<S, OPK>(I, e, cur, nxt, first, acc);
        }
        block_reduce_store<Dots<S>::DD>(acc.s0, acc.c0, acc.s1, acc.c1, part + (size_t)t * 4);
    }
}

// ---------------------------------------------------------------------------
// reduction of the per-tile partials and the moments
// ---------------------------------------------------------------------------
// Block (x, h): dots index idx = step0 + 1 + klo + x of instance h, for x < nk.
__global__ __launch_bounds__(BLOCK) void k_reduce(const Inst *__restrict__ tab, int32_t klo, int32_t nk)
{
    const Inst *I = tab + blockIdx.y;
    if ((int32_t)blockIdx.x >= nk) return;
    const int32_t idx = I->step0 + 1 + klo + (int32_t)blockIdx.x;
    if (idx < 0 || idx > I->K) return;
    const double *p = I->partial + (size_t)(idx % I->pslots) * I->tiles * 4;
    dd a{0.0, 0.0}, b{0.0, 0.0};
    for (uint32_t t = threadIdx.x; t < I->tiles; t += BLOCK) {
        a = dd_add(a, dd{p[(size_t)t * 4 + 0], p[(size_t)t * 4 + 1]});
        b = dd_add(b, dd{p[(size_t)t * 4 + 2], p[(size_t)t * 4 + 3]});
    }
    block_reduce_store<true>(a.hi, a.lo, b.hi, b.lo, I->dots + (size_t)idx * 4);
}

// mu_0 = S_nn[0]/norm, mu_1 = S_nm[1]/norm,
// mu_{2n} = (2 S_nn[n] - S_nn[0])/norm, mu_{2n+1} = (2 S_nm[n+1] - S_nm[1])/norm,
// formed in double-double and rounded once.
__global__ __launch_bounds__(BLOCK) void k_moments(const Inst *__restrict__ tab)
{
    const Inst *I = tab + blockIdx.y;
    const int32_t m = blockIdx.x * BLOCK + threadIdx.x;
    if (m >= I->M) return;
    const double *D = I->dots;
    dd v;
    if (m == 0) {
        v = dd{D[0], D[1]};
    } else if (m == 1) {
        v = dd{D[4 + 2], D[4 + 3]};
    } else if ((m & 1) == 0) {
        const int n = m / 2;
        v = dd_add(dd{2.0 * D[n * 4 + 0], 2.0 * D[n * 4 + 1]}, dd{-D[0], -D[1]});
    } else {
        const int n1 = m / 2 + 1;
        v = dd_add(dd{2.0 * D[n1 * 4 + 2], 2.0 * D[n1 * 4 + 3]}, dd{-D[4 + 2], -D[4 + 3]});
    }
    const dd q = dd_div_d(v, I->norm);
    I->mu[m] = q.hi + q.lo;
}

}  // namespace kpm
