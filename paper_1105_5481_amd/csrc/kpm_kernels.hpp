// Kernels of libkpm for gfx950.
//
// The hot path is the fused recursion step (Eq. (rn) of Zhang et al. 2011):
//     r_{n+1} = 2 H~ r_n - r_{n-1},  written over r_{n-1},
// with the two dot products <r_{n+1}|r_{n+1}> and Re<r_{n+1}|r_n> that the
// doubling identities turn into mu_{2n+2} and mu_{2n+1}, taken from registers
// in the same pass.
//
// Layout.  Vectors are stored site-major: the R vectors (or 2R interleaved
// re/im scalars) of site i are contiguous, padded to a multiple of 16 bytes
// ("chunks").  A thread moves one 16-byte chunk per stream; a wavefront reads
// whole cache lines, and the neighbour of a site is the same chunk of the
// neighbouring site.
//
// March kernels (lattices).  The slowest lattice axis (y in 2D, z in 3D) is
// the march axis; a "plane" is the set of sites with one march coordinate and
// a "column" is one in-plane position.  A thread owns one chunk of one column
// and walks a segment of S planes, keeping the chunk of planes m-1, m, m+1 in
// registers: each vector element of r_n is fetched once per step from HBM
// (plus two halo planes per segment).  In-plane neighbours are read through
// L1/L2 from the adjacent columns, which neighbouring lanes and blocks of the
// same XCD load in the same pass.
//
// Flat kernels (CSR, and lattices on request).  Work is cut into tiles of
// 256*TPT consecutive chunks; every neighbour is loaded through the caches.
//
// Reductions.  Each work item (march: column tile x segment; flat: tile) of a
// step leaves one partial (FP64 sums of its dot products) in a ring of
// per-step slots; a separate kernel sums the partials of a step over the items
// in a fixed order.  Results therefore do not depend on the launch grid or on
// which other instances share the launch.  The blocks of one instance walk
// its items per XCD (block b runs on XCD b mod 8 under round-robin dispatch):
// XCD x owns the x-th eighth of the column tiles (march) or tiles (flat).
#pragma once

#include "kpm_device.hpp"

#define KPM_GLOBAL __attribute__((address_space(1)))

namespace kpm {

enum OpKind { OP_REAL2 = 0, OP_REAL3 = 1, OP_SPIN2 = 2, OP_SPIN3 = 3, OP_CSR_R = 4, OP_CSR_C = 5, OP_COUNT = 6 };
enum { VEC_RADEMACHER = 0, VEC_PHASE = 1, VEC_UNIT = 2 };
enum { MODE_FLAT = 0, MODE_MARCH = 1, MODE_SMALL = 2 };
constexpr int BLOCK = 256;
constexpr uint32_t XCD_MIN_ITEMS = 64;   // below this an instance's items are not split per XCD
constexpr uint32_t NO_INSTANCE = 0xffffffffu;   // block-map entry of an idle block

// One solve inside a launch (device-resident table entry).
struct Inst {
    int32_t opk;
    int32_t has_diag;
    int32_t mode;
    int32_t xcd;       // items split per XCD (0 none, 1 by units, 2 by segments)
    int32_t alt;       // march: odd segments walk downwards
    int32_t nt;        // march: r_{n-1}/r_{n+1} accessed with non-temporal hints
    uint32_t Lx, Ly, Lz, N;
    FastDiv fLx, fLy, fC;
    uint32_t C;        // 16-byte chunks per site
    uint32_t Rs;       // scalars per site (C * W)
    uint32_t nel;      // N * C
    uint32_t tiles;    // work items per step (= partials per step)
    uint32_t nb;       // blocks given to this instance (multiple of 8)
    uint32_t block0;   // first block of this instance in the grid
    uint32_t bstride;  // its blocks are block0, block0 + bstride, ... (1, or 8 to keep them on one XCD)
    int32_t tpt;       // flat: chunks per thread per tile
    uint32_t P, Lm, S, nct, nseg;  // march: plane size, march extent, segment, column tiles, segments
    int32_t cplx;      // data stored as interleaved complex
    int32_t M, K, R, vec;
    int32_t step0;     // recursion step n = step0 + (launch offset k)
    int32_t pslots;    // ring slots of partials
    int32_t tbh;       // temporal blocking: halo sites each side of an x-tile (= steps of the deepest pass)
    int32_t red_lo, red_n;  // dots indices [red_lo, red_lo + red_n) to reduce (k_reduce_ranges)
    uint64_t seed, instance;
    double norm;       // N R (random kinds) or R (unit vectors)
    const void *diag;  // S[N]
    const void *bond;  // S[N][dim][2]: H~_{i, i+e_ax}
    const void *hop;   // S[1]: H~_ij of the real lattice
    const int64_t *row_ptr;
    const int32_t *col;
    const void *val;   // S[nnz] or S[nnz][2]
    void *buf0, *buf1;
    void *tb2, *tb3;   // temporal blocking: buffers 2 and 3 of four (buf0, buf1 are 0 and 1)
    int32_t tbp, tbc;  // ... and which of them hold r_{step0-1}, r_{step0} (batched passes)
    int32_t tbfull, tbrem;  // batched passes of this chunk: tbfull of depth tbh, then one of depth tbrem
    uint32_t tbg;      // 2D temporal blocking: chunk groups per site (a work item covers C / tbg chunks)
    double *partial;   // [pslots][tiles][4]
    double *dots;      // [K+1][4] = (nn.hi, nn.lo, nm.hi, nm.lo)
    double *mu;        // [M]
};

// ---------------------------------------------------------------------------
// global-memory access with a uniform base and a 32-bit (or, for buffers of
// 4 GiB and more, 64-bit) byte offset
// ---------------------------------------------------------------------------
template <typename S, bool WIDE> struct Mem {
    typedef typename V16<S>::T T;
    typedef S S2 __attribute__((ext_vector_type(2)));
    static __device__ __forceinline__ const KPM_GLOBAL char *at(const void *b, uint32_t chunk)
    {
        if (WIDE) return (const KPM_GLOBAL char *)b + ((uint64_t)chunk << 4);
        return (const KPM_GLOBAL char *)b + (chunk << 4);
    }
    static __device__ __forceinline__ T ld(const void *b, uint32_t chunk) { return *(const KPM_GLOBAL T *)at(b, chunk); }
    static __device__ __forceinline__ T ld_nt(const void *b, uint32_t chunk)
    {
        return __builtin_nontemporal_load((const KPM_GLOBAL T *)at(b, chunk));
    }
    static __device__ __forceinline__ void st_nt(void *b, uint32_t chunk, T v)
    {
        __builtin_nontemporal_store(v, (KPM_GLOBAL T *)at(b, chunk));
    }
    // streamed access of r_{n-1} / r_{n+1}: non-temporal (NT) or cached
    template <bool NT> static __device__ __forceinline__ T ld_s(const void *b, uint32_t chunk)
    {
        if (NT) return ld_nt(b, chunk);
        return ld(b, chunk);
    }
    template <bool NT> static __device__ __forceinline__ void st_s(void *b, uint32_t chunk, T v)
    {
        if (NT) st_nt(b, chunk, v);
        else st(b, chunk, v);
    }
    static __device__ __forceinline__ void st(void *b, uint32_t chunk, T v) { *(KPM_GLOBAL T *)at(b, chunk) = v; }
    // element e of an array of S
    static __device__ __forceinline__ S lds(const void *b, uint32_t e)
    {
        if (WIDE) return *(const KPM_GLOBAL S *)((const KPM_GLOBAL char *)b + (uint64_t)e * sizeof(S));
        return *(const KPM_GLOBAL S *)((const KPM_GLOBAL char *)b + e * (uint32_t)sizeof(S));
    }
    // complex element e of an array of S pairs
    static __device__ __forceinline__ S2 ldc(const void *b, uint32_t e)
    {
        if (WIDE) return *(const KPM_GLOBAL S2 *)((const KPM_GLOBAL char *)b + (uint64_t)e * (2 * sizeof(S)));
        return *(const KPM_GLOBAL S2 *)((const KPM_GLOBAL char *)b + e * (uint32_t)(2 * sizeof(S)));
    }
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

// Sum (x0 + x1, x2 + x3) over the wavefront: every lane receives the sums,
// as double-double pairs (x0, x1), (x2, x3) when DD, else in x0 and x2 with
// x1 = x3 = 0.
template <bool DD>
__device__ __forceinline__ void wave_reduce(double &x0, double &x1, double &x2, double &x3)
{
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
}

// The wavefront's sums of (x0 + x1, x2 + x3); lane 0 stores the four doubles
// (hi, lo, hi, lo) at dst.
template <bool DD>
__device__ __forceinline__ void wave_reduce_store(double x0, double x1, double x2, double x3, double *dst)
{
    wave_reduce<DD>(x0, x1, x2, x3);
    if ((threadIdx.x & 63) == 0) {
        dst[0] = x0; dst[1] = x1; dst[2] = x2; dst[3] = x3;
    }
}

// Sum (x0 + x1, x2 + x3) over the block in a fixed order; thread 0 stores
// the four doubles (hi, lo, hi, lo) at dst.
template <bool DD, int NT = BLOCK>
__device__ __forceinline__ void block_reduce_store(double x0, double x1, double x2, double x3, double *dst)
{
    __shared__ double red[NT / 64][4];
    wave_reduce<DD>(x0, x1, x2, x3);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) {
        red[w][0] = x0; red[w][1] = x1; red[w][2] = x2; red[w][3] = x3;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        dd a{red[0][0], red[0][1]}, b{red[0][2], red[0][3]};
#pragma unroll
        for (int k = 1; k < NT / 64; ++k) {
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
// mapping of an instance's blocks to its work items
// ---------------------------------------------------------------------------
// Work items of this instance handled by the block.  An item is (unit, seg)
// with unit a column tile (march) or tile (flat).  Local item index it ->
// seg = sb + it / nu, unit = ub + it % nu, for it = first, first + stride, ...
// below count.  XCD split (block b runs on XCD b mod 8):
//   xcd == 2: XCD x owns segments [x*segs/8, (x+1)*segs/8) of every unit, so a
//             whole plane stays in one L2;
//   xcd == 1: XCD x owns units [x*units/8, (x+1)*units/8) of every segment;
//   xcd == 0: no split.
struct ItemRange {
    uint32_t first, stride, count, ub, nu, sb;
};
__device__ __forceinline__ ItemRange item_range(const Inst &I, uint32_t units, uint32_t segs)
{
    const uint32_t bl = (blockIdx.x - I.block0) / I.bstride;
    ItemRange r;
    r.ub = 0;
    r.nu = units;
    r.sb = 0;
    uint32_t ns = segs;
    if (I.xcd) {
        const uint32_t x8 = bl & 7u;
        if (I.xcd == 2) {
            r.sb = (uint32_t)(((uint64_t)segs * x8) >> 3);
            ns = (uint32_t)(((uint64_t)segs * (x8 + 1)) >> 3) - r.sb;
        } else {
            r.ub = (uint32_t)(((uint64_t)units * x8) >> 3);
            r.nu = (uint32_t)(((uint64_t)units * (x8 + 1)) >> 3) - r.ub;
        }
        r.first = bl >> 3;
        r.stride = I.nb >> 3;
    } else {
        r.first = bl;
        r.stride = I.nb;
    }
    r.count = r.nu * ns;
    return r;
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
// Random phases: xi = e^{i phi}, phi = 2 pi k / 2^30 with k = word >> 34,
// formed as the ordered product (ascending j) of w_j = e^{2 pi i 2^j / 2^30}
// over the set bits of k.  The factors are computed on the host from the
// half-angle recurrence with IEEE operations only and placed in constant
// memory, so the phases are reproducible bit for bit on any IEEE machine.
constexpr int PHASE_BITS = 30;
__constant__ double kpm_phase_w[PHASE_BITS][2];

// The phases of NC vectors at once, k[l] = the top PHASE_BITS bits of their
// words: every lane runs through all PHASE_BITS factors (uniform, so they come
// from scalar loads) and takes the product z * w_j only where bit j of its k is
// set, so the factors multiply in ascending j as defined above.  z starts at 1:
// 1 * w_j gives w_j exactly (w_j has no zero of negative sign), the first
// factor itself, and k = 0 gives 1.
template <int NC>
__device__ __forceinline__ void phase_products(const uint32_t (&k)[NC], double (&zr)[NC], double (&zi)[NC])
{
#pragma unroll
    for (int l = 0; l < NC; ++l) {
        zr[l] = 1.0;
        zi[l] = 0.0;
    }
#pragma unroll 2
    for (int j = 0; j < PHASE_BITS; ++j) {
        const double wr = kpm_phase_w[j][0], wi = kpm_phase_w[j][1];
#pragma unroll
        for (int l = 0; l < NC; ++l) {
            const double tr = zr[l] * wr - zi[l] * wi;
            const double ti = zr[l] * wi + zi[l] * wr;
            const bool set = (k[l] >> j) & 1u;
            zr[l] = set ? tr : zr[l];
            zi[l] = set ? ti : zi[l];
        }
    }
}

// (re, im) of xi_{r,i} given its Philox word.
__device__ __forceinline__ void start_value(int vec, uint64_t word, uint64_t instance, uint32_t N, uint32_t i,
                                            uint32_t r, double &re, double &im)
{
    if (vec == VEC_RADEMACHER) {
        re = (word >> 63) ? -1.0 : 1.0;
        im = 0.0;
    } else if (vec == VEC_PHASE) {
        const uint32_t k[1] = {(uint32_t)(word >> (64 - PHASE_BITS))};
        double zr[1], zi[1];
        phase_products<1>(k, zr, zi);
        re = zr[0];
        im = zi[0];
    } else {
        uint64_t j = (instance + (uint64_t)r) % (uint64_t)N;
        re = (j == (uint64_t)i) ? 1.0 : 0.0;
        im = 0.0;
    }
}

// Chunk c of site i of the start block.
template <typename S>
__device__ __forceinline__ typename V16<S>::T start_chunk(const Inst &I, uint32_t i, uint32_t c)
{
    typedef typename V16<S>::T T;
    constexpr int W = V16<S>::W;
    const uint32_t k0 = c * W;                  // first scalar of the chunk
    const uint32_t r0 = I.cplx ? k0 / 2 : k0;   // first vector of the chunk (all in one Philox block)
    uint64_t w[4] = {0, 0, 0, 0};
    if (I.vec != VEC_UNIT) start_words(I.seed, I.instance, i, r0 / 4, w);
    T v;
    if (I.cplx && I.vec == VEC_PHASE) {
        // the chunk's W / 2 phases in one pass over the factors
        constexpr int NC = W / 2;
        uint32_t k[NC];
        double zr[NC], zi[NC];
#pragma unroll
        for (int l = 0; l < NC; ++l) k[l] = (uint32_t)(w[(r0 + l) & 3] >> (64 - PHASE_BITS));
        phase_products<NC>(k, zr, zi);
#pragma unroll
        for (int l = 0; l < NC; ++l) {
            const bool in = r0 + l < (uint32_t)I.R;
            v[2 * l] = in ? (S)zr[l] : (S)0;
            v[2 * l + 1] = in ? (S)zi[l] : (S)0;
        }
    } else if (I.cplx) {
#pragma unroll
        for (int l = 0; l < W / 2; ++l) {
            const uint32_t r = r0 + l;
            double re = 0.0, im = 0.0;
            if (r < (uint32_t)I.R) start_value(I.vec, w[r & 3], I.instance, I.N, i, r, re, im);
            v[2 * l] = (S)re;
            v[2 * l + 1] = (S)im;
        }
    } else {
#pragma unroll
        for (int l = 0; l < W; ++l) {
            const uint32_t r = r0 + l;
            double re = 0.0, im = 0.0;
            if (r < (uint32_t)I.R) start_value(I.vec, w[r & 3], I.instance, I.N, i, r, re, im);
            v[l] = (S)re;
        }
    }
    return v;
}

// r_0 into buf0 and the partials of <r_0|r_0>, over the same work items as the
// recursion step of the instance's mode.
template <typename S, bool WIDE>
__global__ __launch_bounds__(BLOCK) void k_init(const Inst *__restrict__ tab, const uint32_t *__restrict__ bmap)
{
    typedef Mem<S, WIDE> G;
    const uint32_t h = bmap ? bmap[blockIdx.x] : 0u;
    if (h == NO_INSTANCE) return;
    const Inst I = tab[h];
    if (I.step0 != 0) return;
    double *part = I.partial;   // slot 0
    if (I.mode == MODE_MARCH) {
        const ItemRange ir = item_range(I, I.nct, I.nseg);
        const uint32_t PC = I.P * I.C;
        for (uint32_t it = ir.first; it < ir.count; it += ir.stride) {
            const uint32_t sl = it / ir.nu;
            const uint32_t sg = ir.sb + sl;
            const uint32_t ct = ir.ub + (it - sl * ir.nu);
            const uint32_t e = ct * BLOCK + threadIdx.x;
            Dots<S> acc;
            if (e < PC) {
                const uint32_t p = fdiv(e, I.fC), c = e - p * I.C;
                const uint32_t m0 = sg * I.S, m1 = min(m0 + I.S, I.Lm);
                for (uint32_t m = m0; m < m1; ++m) {
                    const uint32_t i = p + I.P * m;
                    const auto v = start_chunk<S>(I, i, c);
                    G::st(I.buf0, i * I.C + c, v);
                    acc.norm_only(v);
                }
            }
            block_reduce_store<Dots<S>::DD>(acc.s0, acc.c0, acc.s1, acc.c1, part + (size_t)(sg * I.nct + ct) * 4);
        }
    } else {
        const ItemRange ir = item_range(I, I.tiles, 1);
        for (uint32_t it = ir.first; it < ir.count; it += ir.stride) {
            const uint32_t t = ir.ub + it;
            Dots<S> acc;
            for (int u = 0; u < I.tpt; ++u) {
                const uint32_t e = t * (uint32_t)(BLOCK * I.tpt) + (uint32_t)(u * BLOCK) + threadIdx.x;
                if (e < I.nel) {
                    const uint32_t i = fdiv(e, I.fC), c = e - i * I.C;
                    const auto v = start_chunk<S>(I, i, c);
                    G::st(I.buf0, e, v);
                    acc.norm_only(v);
                }
            }
            block_reduce_store<Dots<S>::DD>(acc.s0, acc.c0, acc.s1, acc.c1, part + (size_t)t * 4);
        }
    }
}

// ---------------------------------------------------------------------------
// operator application on one chunk, in the oracle's slot order
// (diagonal, -x, +x, -y, +y[, -z, +z])
// ---------------------------------------------------------------------------
// Real hopping: a = d*v + h*(v_-x) + h*(v_+x) + ...
template <typename S, int NS>
__device__ __forceinline__ typename V16<S>::T apply_real(bool hd, S d, S h, typename V16<S>::T v,
                                                         const typename V16<S>::T (&nb)[NS])
{
    typedef Arith<S> A;
    typename V16<S>::T a;
    if (hd) {
        a = d * v;
        a = A::mac(a, h, nb[0]);
    } else {
        a = h * nb[0];
    }
#pragma unroll
    for (int s = 1; s < NS; ++s) a = A::mac(a, h, nb[s]);
    return a;
}
// Complex hopping: slot s has coefficient (hr[s], hi[s]).
template <typename S, int NS>
__device__ __forceinline__ typename V16<S>::T apply_cplx(bool hd, S d, typename V16<S>::T v,
                                                         const typename V16<S>::T (&nb)[NS], const S (&hr)[NS],
                                                         const S (&hi)[NS])
{
    typedef Arith<S> A;
    constexpr int W = V16<S>::W;
    typename V16<S>::T out;
#pragma unroll
    for (int l = 0; l < W / 2; ++l) {
        S ar, ai;
        if (hd) {
            ar = d * v[2 * l];
            ai = d * v[2 * l + 1];
            A::cmac(ar, ai, hr[0], hi[0], nb[0][2 * l], nb[0][2 * l + 1]);
        } else {
            A::cmul(ar, ai, hr[0], hi[0], nb[0][2 * l], nb[0][2 * l + 1]);
        }
#pragma unroll
        for (int s = 1; s < NS; ++s) A::cmac(ar, ai, hr[s], hi[s], nb[s][2 * l], nb[s][2 * l + 1]);
        out[2 * l] = ar;
        out[2 * l + 1] = ai;
    }
    return out;
}

// ---------------------------------------------------------------------------
// the fused recursion step, march form (lattices)
// ---------------------------------------------------------------------------
template <typename S, int OPK, bool WIDE, bool NT>
__global__ __launch_bounds__(BLOCK) void k_step_march(const Inst *__restrict__ tab,
                                                      const uint32_t *__restrict__ bmap, int32_t k)
{
    typedef typename V16<S>::T T;
    typedef Mem<S, WIDE> G;
    typedef typename Mem<S, WIDE>::S2 S2;
    constexpr bool D3 = (OPK == OP_REAL3 || OPK == OP_SPIN3);
    constexpr bool SPIN = (OPK == OP_SPIN2 || OPK == OP_SPIN3);
    constexpr int DIM = D3 ? 3 : 2;
    constexpr int NS = 2 * DIM;
    const uint32_t h = bmap ? bmap[blockIdx.x] : 0u;
    if (h == NO_INSTANCE) return;
    const Inst I = tab[h];
    const int32_t n = I.step0 + k;
    if (n < 0 || n >= I.K) return;
    const void *cur = (n & 1) ? I.buf1 : I.buf0;
    void *nxt = (n & 1) ? I.buf0 : I.buf1;
    const bool first = (n == 0);
    const bool hd = I.has_diag;
    S hop = 0;
    if (!SPIN) hop = G::lds(I.hop, 0);
    double *part = I.partial + (size_t)((n + 1) % I.pslots) * I.tiles * 4;
    const uint32_t C = I.C, P = I.P, Lx = I.Lx, Ly = I.Ly, Lm = I.Lm;
    const uint32_t PC = P * C;
    const ItemRange ir = item_range(I, I.nct, I.nseg);
    for (uint32_t it = ir.first; it < ir.count; it += ir.stride) {
        const uint32_t sl = it / ir.nu;
        const uint32_t sg = ir.sb + sl;
        const uint32_t ct = ir.ub + (it - sl * ir.nu);
        const uint32_t e = ct * BLOCK + threadIdx.x;
        Dots<S> acc;
        if (e < PC) {
            const uint32_t p = fdiv(e, I.fC), c = e - p * C;
            uint32_t x = p, y = 0;
            if constexpr (D3) {
                y = fdiv(p, I.fLx);
                x = p - y * Lx;
            }
            const uint32_t pxm = (x == 0) ? p + (Lx - 1) : p - 1;
            const uint32_t pxp = (x == Lx - 1) ? p - (Lx - 1) : p + 1;
            uint32_t pym = 0, pyp = 0;
            if constexpr (D3) {
                pym = (y == 0) ? p + (Ly - 1) * Lx : p - Lx;
                pyp = (y == Ly - 1) ? p - (Ly - 1) * Lx : p + Lx;
            }
            const uint32_t m0 = sg * I.S, m1 = min(m0 + I.S, Lm);
            // Odd segments march downwards, so that two adjacent segments reach
            // their common boundary planes at about the same time and the second
            // read of a halo plane hits in L2.
            const bool down = I.alt && (sg & 1u) != 0;
            const uint32_t mfirst = down ? m1 - 1 : m0;
            const uint32_t mbefore = down ? ((m1 == Lm) ? 0 : m1) : ((m0 == 0) ? Lm - 1 : m0 - 1);
            // window: vb = plane behind (in march order), v0 = current plane
            T vb = G::ld(cur, (p + P * mbefore) * C + c);
            T v0 = G::ld(cur, (p + P * mfirst) * C + c);
            // march-axis bond linking plane mbefore and mfirst (H~_{(m-1), m} stored at plane m-1)
            S2 bb = {0, 0};
            if (SPIN) bb = G::ldc(I.bond, (p + P * (down ? mfirst : mbefore)) * DIM + (DIM - 1));
            for (uint32_t s_ = 0; s_ < m1 - m0; ++s_) {
                const uint32_t m = down ? mfirst - s_ : mfirst + s_;
                const uint32_t ma = down ? ((m == 0) ? Lm - 1 : m - 1) : ((m + 1 == Lm) ? 0 : m + 1);  // plane ahead
                const uint32_t i = p + P * m;
                const uint32_t ch = i * C + c;
                const T va = G::ld(cur, (p + P * ma) * C + c);
                T nb[NS];
                nb[0] = G::ld(cur, (pxm + P * m) * C + c);
                nb[1] = G::ld(cur, (pxp + P * m) * C + c);
                if constexpr (D3) {
                    nb[2] = G::ld(cur, (pym + P * m) * C + c);
                    nb[3] = G::ld(cur, (pyp + P * m) * C + c);
                }
                // slots -march, +march in the fixed order
                nb[NS - 2] = down ? va : vb;
                nb[NS - 1] = down ? vb : va;
                T prev;
                if (!first) prev = G::template ld_s<NT>(nxt, ch);
                const S d = hd ? G::lds(I.diag, i) : (S)0;
                T out;
                if (!SPIN) {
                    out = apply_real<S, NS>(hd, d, hop, v0, nb);
                } else {
                    S hr[NS], hi[NS];
                    const S2 bxm = G::ldc(I.bond, (pxm + P * m) * DIM + 0);
                    const S2 bxp = G::ldc(I.bond, i * DIM + 0);
                    hr[0] = bxm[0]; hi[0] = -bxm[1];
                    hr[1] = bxp[0]; hi[1] = bxp[1];
                    if constexpr (D3) {
                        const S2 bym = G::ldc(I.bond, (pym + P * m) * DIM + 1);
                        const S2 byp = G::ldc(I.bond, i * DIM + 1);
                        hr[2] = bym[0]; hi[2] = -bym[1];
                        hr[3] = byp[0]; hi[3] = byp[1];
                    }
                    // the other march-axis bond: H~_{m, m+1} (up) lives at plane m,
                    // H~_{m-1, m} (down) at plane m-1 = the plane ahead
                    const S2 ba = G::ldc(I.bond, (p + P * (down ? ma : m)) * DIM + (DIM - 1));
                    const S2 bminus = down ? ba : bb;   // H~_{m-1,m}: conjugated for slot -march
                    const S2 bplus = down ? bb : ba;    // H~_{m,m+1}
                    hr[NS - 2] = bminus[0]; hi[NS - 2] = -bminus[1];
                    hr[NS - 1] = bplus[0]; hi[NS - 1] = bplus[1];
                    out = apply_cplx<S, NS>(hd, d, v0, nb, hr, hi);
                    bb = ba;
                }
                if (!first) out = (S)2 * out - prev;
                G::template st_s<NT>(nxt, ch, out);
                acc.add(out, v0);
                vb = v0;
                v0 = va;
            }
        }
        block_reduce_store<Dots<S>::DD>(acc.s0, acc.c0, acc.s1, acc.c1, part + (size_t)(sg * I.nct + ct) * 4);
    }
}

// ---------------------------------------------------------------------------
// the fused recursion step, flat form (CSR; lattices on request)
// ---------------------------------------------------------------------------
template <typename S, int OPK, bool WIDE>
__device__ __forceinline__ void flat_elem(const Inst &I, uint32_t e, const void *cur, void *nxt, bool first, S hop,
                                          Dots<S> &acc)
{
    typedef typename V16<S>::T T;
    typedef Mem<S, WIDE> G;
    typedef typename Mem<S, WIDE>::S2 S2;
    typedef Arith<S> A;
    constexpr int W = V16<S>::W;
    const uint32_t C = I.C;
    const uint32_t i = fdiv(e, I.fC);
    const uint32_t c = e - i * C;
    const T v = G::ld(cur, e);
    T out;
    if constexpr (OPK <= OP_SPIN3) {
        constexpr bool D3 = (OPK == OP_REAL3 || OPK == OP_SPIN3);
        constexpr bool SPIN = (OPK == OP_SPIN2 || OPK == OP_SPIN3);
        constexpr int DIM = D3 ? 3 : 2;
        constexpr int NS = 2 * DIM;
        const uint32_t Lx = I.Lx, Ly = I.Ly;
        const uint32_t yq = fdiv(i, I.fLx);
        const uint32_t x = i - yq * Lx;
        uint32_t y = yq, z = 0;
        if constexpr (D3) {
            z = fdiv(yq, I.fLy);
            y = yq - z * Ly;
        }
        uint32_t nbi[NS];
        nbi[0] = (x == 0) ? i + (Lx - 1) : i - 1;
        nbi[1] = (x == Lx - 1) ? i - (Lx - 1) : i + 1;
        nbi[2] = (y == 0) ? i + (Ly - 1) * Lx : i - Lx;
        nbi[3] = (y == Ly - 1) ? i - (Ly - 1) * Lx : i + Lx;
        if constexpr (D3) {
            const uint32_t Pz = Lx * Ly, Lz = I.Lz;
            nbi[4] = (z == 0) ? i + (Lz - 1) * Pz : i - Pz;
            nbi[5] = (z == Lz - 1) ? i - (Lz - 1) * Pz : i + Pz;
        }
        T nb[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s) nb[s] = G::ld(cur, nbi[s] * C + c);
        const bool hd = I.has_diag;
        const S d = hd ? G::lds(I.diag, i) : (S)0;
        if (!SPIN) {
            out = apply_real<S, NS>(hd, d, hop, v, nb);
        } else {
            S hr[NS], hi[NS];
#pragma unroll
            for (int ax = 0; ax < DIM; ++ax) {
                const S2 bm = G::ldc(I.bond, nbi[2 * ax] * DIM + ax);
                const S2 bp = G::ldc(I.bond, i * DIM + ax);
                hr[2 * ax] = bm[0]; hi[2 * ax] = -bm[1];
                hr[2 * ax + 1] = bp[0]; hi[2 * ax + 1] = bp[1];
            }
            out = apply_cplx<S, NS>(hd, d, v, nb, hr, hi);
        }
    } else {
        // CSR: the diagonal d_i first, then the off-diagonal entries in stored order
        const int64_t kb = I.row_ptr[i], ke = I.row_ptr[i + 1];
        const S d = G::lds(I.diag, i);
        T a;
#pragma unroll
        for (int l = 0; l < W; ++l) a[l] = d * v[l];
        for (int64_t kk = kb; kk < ke; ++kk) {
            const uint32_t jj = (uint32_t)I.col[kk];
            if (jj == i) continue;
            const T vj = G::ld(cur, jj * C + c);
            if constexpr (OPK == OP_CSR_R) {
                a = A::mac(a, ((const S *)I.val)[kk], vj);
            } else {
                const S hr = ((const S *)I.val)[2 * kk], hi = ((const S *)I.val)[2 * kk + 1];
#pragma unroll
                for (int l = 0; l < W / 2; ++l) {
                    S ar = a[2 * l], ai = a[2 * l + 1];
                    A::cmac(ar, ai, hr, hi, vj[2 * l], vj[2 * l + 1]);
                    a[2 * l] = ar;
                    a[2 * l + 1] = ai;
                }
            }
        }
        out = a;
    }
    if (!first) {
        const T p = G::ld_nt(nxt, e);
        out = (S)2 * out - p;
    }
    G::st_nt(nxt, e, out);
    acc.add(out, v);
}

template <typename S, int OPK, bool WIDE>
__global__ __launch_bounds__(BLOCK) void k_step_flat(const Inst *__restrict__ tab, const uint32_t *__restrict__ bmap,
                                                     int32_t k)
{
    const uint32_t h = bmap ? bmap[blockIdx.x] : 0u;
    if (h == NO_INSTANCE) return;
    const Inst I = tab[h];
    const int32_t n = I.step0 + k;
    if (n < 0 || n >= I.K) return;
    const void *cur = (n & 1) ? I.buf1 : I.buf0;
    void *nxt = (n & 1) ? I.buf0 : I.buf1;
    const bool first = (n == 0);
    S hop = 0;
    if (OPK == OP_REAL2 || OPK == OP_REAL3) hop = Mem<S, WIDE>::lds(I.hop, 0);
    double *part = I.partial + (size_t)((n + 1) % I.pslots) * I.tiles * 4;
    const ItemRange ir = item_range(I, I.tiles, 1);
    for (uint32_t it = ir.first; it < ir.count; it += ir.stride) {
        const uint32_t t = ir.ub + it;
        Dots<S> acc;
        for (int u = 0; u < I.tpt; ++u) {
            const uint32_t e = t * (uint32_t)(BLOCK * I.tpt) + (uint32_t)(u * BLOCK) + threadIdx.x;
            if (e < I.nel) flat_elem<S, OPK, WIDE>(I, e, cur, nxt, first, hop, acc);
        }
        block_reduce_store<Dots<S>::DD>(acc.s0, acc.c0, acc.s1, acc.c1, part + (size_t)t * 4);
    }
}

// ---------------------------------------------------------------------------
// the whole solve of a small instance inside one workgroup
// ---------------------------------------------------------------------------
// Both vector blocks live in LDS (2 * N * C * 16 bytes <= the LDS of one CU),
// so the recursion never touches HBM; one block per instance, all steps in one
// launch, one block barrier between steps.  The per-step dots are summed per
// wave only: partial slot n + 1 holds SMALL_WAVES entries (a block-wide sum
// each step, whose last part one thread does alone, took about two thirds of
// the solve), reduced by k_reduce after the launch.
constexpr int SMALL_BLOCK = 1024;
constexpr int SMALL_WAVES = SMALL_BLOCK / 64;

template <typename S, int OPK>
__device__ __forceinline__ typename V16<S>::T small_elem(const Inst &I, uint32_t e, const typename V16<S>::T *cur,
                                                         S hop)
{
    typedef typename V16<S>::T T;
    typedef Mem<S, false> G;
    typedef typename Mem<S, false>::S2 S2;
    typedef Arith<S> A;
    constexpr int W = V16<S>::W;
    const uint32_t C = I.C;
    const uint32_t i = fdiv(e, I.fC);
    const uint32_t c = e - i * C;
    const T v = cur[e];
    T out;
    if constexpr (OPK <= OP_SPIN3) {
        constexpr bool D3 = (OPK == OP_REAL3 || OPK == OP_SPIN3);
        constexpr bool SPIN = (OPK == OP_SPIN2 || OPK == OP_SPIN3);
        constexpr int DIM = D3 ? 3 : 2;
        constexpr int NS = 2 * DIM;
        const uint32_t Lx = I.Lx, Ly = I.Ly;
        const uint32_t yq = fdiv(i, I.fLx);
        const uint32_t x = i - yq * Lx;
        uint32_t y = yq, z = 0;
        if constexpr (D3) {
            z = fdiv(yq, I.fLy);
            y = yq - z * Ly;
        }
        uint32_t nbi[NS];
        nbi[0] = (x == 0) ? i + (Lx - 1) : i - 1;
        nbi[1] = (x == Lx - 1) ? i - (Lx - 1) : i + 1;
        nbi[2] = (y == 0) ? i + (Ly - 1) * Lx : i - Lx;
        nbi[3] = (y == Ly - 1) ? i - (Ly - 1) * Lx : i + Lx;
        if constexpr (D3) {
            const uint32_t Pz = Lx * Ly, Lz = I.Lz;
            nbi[4] = (z == 0) ? i + (Lz - 1) * Pz : i - Pz;
            nbi[5] = (z == Lz - 1) ? i - (Lz - 1) * Pz : i + Pz;
        }
        T nb[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s) nb[s] = cur[nbi[s] * C + c];
        const bool hd = I.has_diag;
        const S d = hd ? G::lds(I.diag, i) : (S)0;
        if (!SPIN) {
            out = apply_real<S, NS>(hd, d, hop, v, nb);
        } else {
            S hr[NS], hi[NS];
#pragma unroll
            for (int ax = 0; ax < DIM; ++ax) {
                const S2 bm = G::ldc(I.bond, nbi[2 * ax] * DIM + ax);
                const S2 bp = G::ldc(I.bond, i * DIM + ax);
                hr[2 * ax] = bm[0]; hi[2 * ax] = -bm[1];
                hr[2 * ax + 1] = bp[0]; hi[2 * ax + 1] = bp[1];
            }
            out = apply_cplx<S, NS>(hd, d, v, nb, hr, hi);
        }
    } else {
        const int64_t kb = I.row_ptr[i], ke = I.row_ptr[i + 1];
        const S d = G::lds(I.diag, i);
        T a;
#pragma unroll
        for (int l = 0; l < W; ++l) a[l] = d * v[l];
        for (int64_t kk = kb; kk < ke; ++kk) {
            const uint32_t jj = (uint32_t)I.col[kk];
            if (jj == i) continue;
            const T vj = cur[jj * C + c];
            if constexpr (OPK == OP_CSR_R) {
                a = A::mac(a, ((const S *)I.val)[kk], vj);
            } else {
                const S hr = ((const S *)I.val)[2 * kk], hi = ((const S *)I.val)[2 * kk + 1];
#pragma unroll
                for (int l = 0; l < W / 2; ++l) {
                    S ar = a[2 * l], ai = a[2 * l + 1];
                    A::cmac(ar, ai, hr, hi, vj[2 * l], vj[2 * l + 1]);
                    a[2 * l] = ar;
                    a[2 * l + 1] = ai;
                }
            }
        }
        out = a;
    }
    return out;
}

template <typename S, int OPK>
__global__ __launch_bounds__(SMALL_BLOCK) void k_solve_small(const Inst *__restrict__ tab)
{
    typedef typename V16<S>::T T;
    extern __shared__ __align__(16) char kpm_lds[];
    const Inst I = tab[blockIdx.x];
    T *b0 = reinterpret_cast<T *>(kpm_lds);
    T *b1 = b0 + I.nel;
    S hop = 0;
    if (OPK == OP_REAL2 || OPK == OP_REAL3) hop = Mem<S, false>::lds(I.hop, 0);
    const uint32_t w = threadIdx.x >> 6;
    {
        Dots<S> acc;
        for (uint32_t e = threadIdx.x; e < I.nel; e += SMALL_BLOCK) {
            const uint32_t i = fdiv(e, I.fC), c = e - i * I.C;
            const T v = start_chunk<S>(I, i, c);
            b0[e] = v;
            acc.norm_only(v);
        }
        wave_reduce_store<Dots<S>::DD>(acc.s0, acc.c0, acc.s1, acc.c1, I.partial + (size_t)w * 4);
    }
    __syncthreads();   // r_0 complete
    for (int32_t n = 0; n < I.K; ++n) {
        const T *cur = (n & 1) ? b1 : b0;
        T *nxt = (n & 1) ? b0 : b1;
        Dots<S> acc;
        for (uint32_t e = threadIdx.x; e < I.nel; e += SMALL_BLOCK) {
            T out = small_elem<S, OPK>(I, e, cur, hop);
            if (n > 0) out = (S)2 * out - nxt[e];
            nxt[e] = out;
            acc.add(out, cur[e]);
        }
        wave_reduce_store<Dots<S>::DD>(acc.s0, acc.c0, acc.s1, acc.c1,
                                       I.partial + ((size_t)(n + 1) * SMALL_WAVES + w) * 4);
        // step n's LDS writes before step n + 1 reads them, and its reads before they are overwritten
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// reduction of the per-item partials and the moments
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

// Block (x, h): dots index red_lo + x of instance h, for x < red_n.
__global__ __launch_bounds__(BLOCK) void k_reduce_ranges(const Inst *__restrict__ tab)
{
    const Inst *I = tab + blockIdx.y;
    if ((int32_t)blockIdx.x >= I->red_n) return;
    const int32_t idx = I->red_lo + (int32_t)blockIdx.x;
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
