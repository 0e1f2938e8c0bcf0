// The dense-H recursion (the paper's own kernel design, Sec. III and the
// H_SIZE experiments of Sec. IV): H~ is a dense D x D real matrix and one
// recursion step over the R vectors is the product H~ V_n (D x D times D x R),
// a dense FP64 contraction, followed by V_{n+1} = 2 H~ V_n - V_{n-1} and the
// two dot products of the doubling identities.
//
// Layout (all FP64, row-major, zero padded): H~ is Dp x Dp and every vector
// block Dp x Rp, Dp and Rp multiples of 64, so padded rows and columns stay
// exactly zero through the recursion and add nothing to the dots.
//
// One workgroup (4 waves) computes a 64 x 64 (or 64 x 32) block of H~ V_n
// with the FP64 matrix instruction v_mfma_f64_16x16x4 (each wave a quarter of
// 2 x 2 or 2 x 1 instruction tiles), staging 64 x 16 slices of H~ and 16 x 64
// (16 x 32) slices of V_n
// through LDS, and finishes the block in registers: the recursion update,
// the store of V_{n+1} over V_{n-1}, and the per-block double-double partial
// sums of <V_{n+1}|V_{n+1}> and <V_{n+1}|V_n>.
//
// Lane layout of v_mfma_f64_16x16x4 (measured on gfx950): lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16] and receives D[4 v + l / 16][l % 16]
// in element v of its 4-vector.
#pragma once

namespace kpm {

constexpr int DN_TILE = 64;     // output block edge
constexpr int DN_KT = 16;       // K slice staged per iteration
typedef double dn_d4 __attribute__((ext_vector_type(4)));

// H~ = (H - b I)/a into the padded Dp x Dp array (rows/cols >= D are zero);
// the same operations as the CSR operator build: (H_ii - b)/a on the
// diagonal, H_ij/a off it.
__global__ __launch_bounds__(256) void k_dense_scale(const double *__restrict__ H, uint32_t D, uint32_t Dp, double a,
                                                     double b, double *__restrict__ Ht)
{
    const uint64_t e = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= (uint64_t)Dp * Dp) return;
    const uint32_t i = (uint32_t)(e / Dp), j = (uint32_t)(e % Dp);
    double v = 0.0;
    if (i < D && j < D) {
        const double h = H[(uint64_t)i * D + j];
        v = (i == j) ? (h - b) / a : h / a;
    }
    Ht[e] = v;
}

// V_0 = xi (R real start vectors of kind vec, column r = vector r) over the
// 64 x tn output tiles of the step kernel, with the partials of <V_0|V_0>
// (slot 0).
__global__ __launch_bounds__(256) void k_dense_init(uint32_t D, uint32_t Dp, uint32_t R, uint32_t Rp, int vec,
                                                    uint64_t seed, uint64_t instance, uint32_t tn,
                                                    double *__restrict__ V, double *__restrict__ part)
{
    const uint32_t tiles_r = Rp / tn;
    const uint32_t i0 = (blockIdx.x / tiles_r) * DN_TILE, r0 = (blockIdx.x % tiles_r) * tn;
    double s = 0.0, c = 0.0;
    for (uint32_t q = threadIdx.x; q < DN_TILE * tn; q += 256) {
        const uint32_t i = i0 + q / tn, r = r0 + q % tn;
        double re = 0.0, im = 0.0;
        if (i < D && r < R) {
            uint64_t w[4] = {0, 0, 0, 0};
            if (vec != VEC_UNIT) start_words(seed, instance, i, r / 4, w);
            start_value(vec, w[r & 3], instance, D, i, r, re, im);
        }
        V[(uint64_t)i * Rp + r] = re;
        dot2_acc(s, c, re, re);
    }
    block_reduce_store<true>(s, c, 0.0, 0.0, part + (size_t)blockIdx.x * 4);
}

// One recursion step: next = H~ cur (FIRST) or 2 H~ cur - next, and the
// partials of <next|next>, <next|cur> for the dots index of this step.
// The block computes 64 x TN outputs with its 4 waves in 2 x 2 quarters of
// 32 x TN/2 (TN = 64, or 32 to give small products twice the blocks).
// The register budget is capped for 5 waves per SIMD: at the compiler's own
// choice (99 VGPRs + 32 AGPRs, 3 waves) the matrix pipe idled a third of the
// time (D = 4096: 50.7 TFLOP/s; capped: 61.6, no spills).  (Blocks of 128
// rows, every A value feeding 4 instructions, measured slower: 45.5 vs 52
// TFLOP/s at D = 4096.)
template <bool FIRST, int TN>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5))) void k_dense_step(
    const double *__restrict__ Ht, const double *__restrict__ cur, double *__restrict__ next, uint32_t Dp, uint32_t Rp,
    double *__restrict__ part)
{
    constexpr int WC = TN / 2;                       // columns per wave
    constexpr int NP = 2, NQ = WC / 16;              // instruction tiles per wave
    constexpr int AL = DN_TILE * DN_KT / 256;        // A values staged per thread per slice
    constexpr int BL = DN_KT * TN / 256;             // B values staged per thread per slice
    __shared__ double As[DN_TILE][DN_KT + 1];
    __shared__ double Bs[DN_KT][TN + 2];
    const uint32_t tiles_r = Rp / TN;
    const uint32_t i0 = (blockIdx.x / tiles_r) * DN_TILE, r0 = (blockIdx.x % tiles_r) * TN;
    const int t = threadIdx.x, l = t & 63, w = t >> 6;
    const int wr = (w >> 1) * 32, wc = (w & 1) * WC;
    const int lr = l & 15, lk = l >> 4;
    dn_d4 acc[NP][NQ];
#pragma unroll
    for (int p = 0; p < NP; ++p)
#pragma unroll
        for (int q = 0; q < NQ; ++q) acc[p][q] = dn_d4{0.0, 0.0, 0.0, 0.0};
    // the slices H~[i0:i0+64, k0:k0+16] and cur[k0:k0+16, r0:r0+TN]; the next
    // slice is loaded into registers while the matrix instructions work on the
    // current one in LDS
    double ra[AL], rb[BL];
#pragma unroll
    for (int u = 0; u < AL; ++u) {
        const int q = t + 256 * u;
        ra[u] = Ht[(uint64_t)(i0 + q / DN_KT) * Dp + (q % DN_KT)];
    }
#pragma unroll
    for (int u = 0; u < BL; ++u) {
        const int q = t + 256 * u;
        rb[u] = cur[(uint64_t)(q / TN) * Rp + r0 + (q % TN)];
    }
    for (uint32_t k0 = 0; k0 < Dp; k0 += DN_KT) {
#pragma unroll
        for (int u = 0; u < AL; ++u) {
            const int q = t + 256 * u;
            As[q / DN_KT][q % DN_KT] = ra[u];
        }
#pragma unroll
        for (int u = 0; u < BL; ++u) {
            const int q = t + 256 * u;
            Bs[q / TN][q % TN] = rb[u];
        }
        __syncthreads();
        if (k0 + DN_KT < Dp) {
#pragma unroll
            for (int u = 0; u < AL; ++u) {
                const int q = t + 256 * u;
                ra[u] = Ht[(uint64_t)(i0 + q / DN_KT) * Dp + k0 + DN_KT + (q % DN_KT)];
            }
#pragma unroll
            for (int u = 0; u < BL; ++u) {
                const int q = t + 256 * u;
                rb[u] = cur[(uint64_t)(k0 + DN_KT + q / TN) * Rp + r0 + (q % TN)];
            }
        }
#pragma unroll
        for (int kk = 0; kk < DN_KT; kk += 4) {
            double av[NP], bv[NQ];
#pragma unroll
            for (int p = 0; p < NP; ++p) av[p] = As[wr + 16 * p + lr][kk + lk];
#pragma unroll
            for (int q = 0; q < NQ; ++q) bv[q] = Bs[kk + lk][wc + 16 * q + lr];
#pragma unroll
            for (int p = 0; p < NP; ++p)
#pragma unroll
                for (int q = 0; q < NQ; ++q) acc[p][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[p], bv[q], acc[p][q], 0, 0, 0);
        }
        __syncthreads();
    }
    double s0 = 0.0, c0 = 0.0, s1 = 0.0, c1 = 0.0;
#pragma unroll
    for (int p = 0; p < NP; ++p)
#pragma unroll
        for (int q = 0; q < NQ; ++q)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const uint32_t i = i0 + wr + 16 * p + 4 * v + lk;
                const uint32_t r = r0 + wc + 16 * q + lr;
                const uint64_t o = (uint64_t)i * Rp + r;
                double out = acc[p][q][v];
                if (!FIRST) out = 2.0 * out - next[o];
                next[o] = out;
                dot2_acc(s0, c0, out, out);
                dot2_acc(s1, c1, out, cur[o]);
            }
    block_reduce_store<true>(s0, c0, s1, c1, part + (size_t)blockIdx.x * 4);
}

// ---------------------------------------------------------------------------
// small H~ (D <= 128): the whole recursion on chip, one launch
// ---------------------------------------------------------------------------
// Each block owns a 16-column slab of the vectors for all steps (Dp = 16 NW):
// wave w computes rows 16w .. 16w + 15 of H~ V_n with Dp/4 matrix
// instructions, whose A operands (the Dp/4 values of H~ a lane supplies) it
// loads once into registers and keeps for the whole solve; the 4 results a
// lane receives (rows 16w + 4v + l/16, column l % 16) are exactly the
// B-operand values the same lane supplies for those rows in the next step, so
// r_{n-1}, r_n and r_{n+1} stay in registers and only the slab of r_n is
// shared through LDS.  H~ must be symmetric: the A operand H~[i][k] is read as
// H~[k][i] (consecutive addresses across a wave).  The products run as 4
// independent accumulation chains.  The per-step dot partials are summed per
// wave only (no block-wide step) and go to slot n + 1 of `part`
// ([K + 1][blocks][NW][4]).

template <int NW>
__global__ __launch_bounds__(64 * NW) void k_dense_resident(const double *__restrict__ Ht, uint32_t D, uint32_t R,
                                                            int vec, uint64_t seed, uint64_t instance, int32_t K,
                                                            double *__restrict__ part)
{
    extern __shared__ double lds[];
    constexpr uint32_t Dp = 16 * NW;
    double *Vs = lds;              // Dp x 16
    const int t = threadIdx.x, l = t & 63, w = t >> 6;
    const int lr = l & 15, lk = l >> 4;
    const uint32_t nblk = gridDim.x;
    const uint32_t col = blockIdx.x * 16 + lr;
    double ha[Dp / 4];   // this lane's A operands: H~[4 s + l/16][16 w + l % 16]
#pragma unroll
    for (uint32_t s = 0; s < Dp / 4; ++s) ha[s] = Ht[(4 * s + lk) * Dp + 16 * w + lr];
    double cur[4], prev[4] = {0.0, 0.0, 0.0, 0.0};
    double s0 = 0.0, e0 = 0.0;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const uint32_t i = 16 * w + 4 * v + lk;
        double re = 0.0, im = 0.0;
        if (i < D && col < R) {
            uint64_t wd[4] = {0, 0, 0, 0};
            if (vec != VEC_UNIT) start_words(seed, instance, i, col / 4, wd);
            start_value(vec, wd[col & 3], instance, D, i, col, re, im);
        }
        cur[v] = re;
        Vs[i * 16 + lr] = re;
        dot2_acc(s0, e0, re, re);
    }
    const size_t wslot = (size_t)blockIdx.x * NW + w;   // this wave's partial within a slot
    wave_reduce_store<true>(s0, e0, 0.0, 0.0, part + wslot * 4);
    __syncthreads();
    for (int32_t n = 0; n < K; ++n) {
        dn_d4 acc[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[c] = dn_d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (uint32_t s = 0; s < Dp / 4; s += 4) {
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const uint32_t k = 4 * (s + c) + lk;
                acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(ha[s + c], Vs[k * 16 + lr], acc[c], 0, 0, 0);
            }
        }
        __syncthreads();   // every wave has read the slab of r_n
        double x0 = 0.0, y0 = 0.0, x1 = 0.0, y1 = 0.0;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            double out = (acc[0][v] + acc[1][v]) + (acc[2][v] + acc[3][v]);
            if (n > 0) out = 2.0 * out - prev[v];
            dot2_acc(x0, y0, out, out);
            dot2_acc(x1, y1, out, cur[v]);
            prev[v] = cur[v];
            cur[v] = out;
            Vs[(16 * w + 4 * v + lk) * 16 + lr] = out;
        }
        wave_reduce_store<true>(x0, y0, x1, y1, part + ((size_t)(n + 1) * nblk * NW + wslot) * 4);
        __syncthreads();   // the slab of r_{n+1} is complete
    }
}

}  // namespace kpm
