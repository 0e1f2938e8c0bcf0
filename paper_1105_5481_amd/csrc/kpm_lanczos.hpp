// Lanczos estimate of the spectral interval of H~ (FP64).
//
// The rescaling H~ = (H - b)/a of Sec. II-A needs an interval that encloses
// the spectrum; Gershgorin's discs always do but can be loose (spin hopping,
// disorder).  The Lanczos three-term process (Golub and Van Loan, Matrix
// Computations, Sec. 10.1) gives Ritz values that converge to the extreme
// eigenvalues from inside; padded by their residual bounds and a relative
// margin, and clipped to Gershgorin, they give a tighter interval.
//
// One start vector in the solve layout with R = 1: one 16-byte chunk per site
// holding (re, im) for a complex operator or (value, 0) for a real one.
//   v_0 = xi / ||xi||;  for j = 0, 1, ...:
//     u = H~ v_j,  alpha_j = Re <v_j|u>,
//     w = (u - alpha_j v_j) - beta_{j-1} v_{j-1}   (last term absent for j = 0),
//     beta_j = ||w||,  v_{j+1} = w / beta_j        (0 if beta_j = 0)
// The scalars stay on the device, in the instance's dots array, as
// double-double sums (each used as its rounded high part):
//   index 0       <xi|xi>
//   index 2j + 1  (||u||^2, Re<u|v_j>)   alpha_j = the second sum
//   index 2j + 2  (||w||^2, 0)           beta_j = sqrt(the first sum)
#pragma once

namespace kpm {

constexpr int LZ_KMAX = 512;       // Lanczos steps per call (LDS of the tridiagonal solve)
constexpr double LZ_BREAKDOWN = 1e-12;

// u = H~ v_j and the partial sums of ||u||^2 and Re<u|v_j> (dots index idx).
template <int OPK, bool WIDE>
__global__ __launch_bounds__(BLOCK) void k_lz_matvec(const Inst *__restrict__ tab, const void *v, void *u,
                                                     int32_t idx)
{
    const Inst I = tab[0];
    double hop = 0.0;
    if (OPK == OP_REAL2 || OPK == OP_REAL3) hop = Mem<double, WIDE>::lds(I.hop, 0);
    double *part = I.partial + (size_t)(idx % I.pslots) * I.tiles * 4;
    const ItemRange ir = item_range(I, I.tiles, 1);
    for (uint32_t it = ir.first; it < ir.count; it += ir.stride) {
        const uint32_t t = ir.ub + it;
        Dots<double> acc;
        for (int q = 0; q < I.tpt; ++q) {
            const uint32_t e = t * (uint32_t)(BLOCK * I.tpt) + (uint32_t)(q * BLOCK) + threadIdx.x;
            if (e < I.nel) flat_elem<double, OPK, WIDE>(I, e, v, u, true, hop, acc);
        }
        block_reduce_store<true>(acc.s0, acc.c0, acc.s1, acc.c1, part + (size_t)t * 4);
    }
}

// w = (u - alpha_j v_j) - beta_{j-1} v_{j-1}, written over v_{j-1}, and the
// partial sums of ||w||^2 (dots index 2j + 2).
template <bool WIDE>
__global__ __launch_bounds__(BLOCK) void k_lz_update(const Inst *__restrict__ tab, const void *u, const void *v,
                                                     void *vp, int32_t j)
{
    typedef Mem<double, WIDE> G;
    typedef V16<double>::T T;
    const Inst I = tab[0];
    const double al = I.dots[(size_t)(2 * j + 1) * 4 + 2];
    const double be = j > 0 ? sqrt(I.dots[(size_t)(2 * j) * 4 + 0]) : 0.0;
    double *part = I.partial + (size_t)((2 * j + 2) % I.pslots) * I.tiles * 4;
    const ItemRange ir = item_range(I, I.tiles, 1);
    for (uint32_t it = ir.first; it < ir.count; it += ir.stride) {
        const uint32_t t = ir.ub + it;
        Dots<double> acc;
        for (int q = 0; q < I.tpt; ++q) {
            const uint32_t e = t * (uint32_t)(BLOCK * I.tpt) + (uint32_t)(q * BLOCK) + threadIdx.x;
            if (e < I.nel) {
                const T uu = G::ld(u, e), vv = G::ld(v, e);
                T w;
#pragma unroll
                for (int l = 0; l < 2; ++l) w[l] = uu[l] - al * vv[l];
                if (j > 0) {
                    const T pp = G::ld(vp, e);
#pragma unroll
                    for (int l = 0; l < 2; ++l) w[l] = w[l] - be * pp[l];
                }
                G::st(vp, e, w);
                acc.norm_only(w);
            }
        }
        block_reduce_store<true>(acc.s0, acc.c0, 0.0, 0.0, part + (size_t)t * 4);
    }
}

// x = x / sqrt(first sum of dots index idx) (x = 0 if that sum is 0).
template <bool WIDE>
__global__ __launch_bounds__(BLOCK) void k_lz_scale(const Inst *__restrict__ tab, void *x, int32_t idx)
{
    typedef Mem<double, WIDE> G;
    typedef V16<double>::T T;
    const Inst I = tab[0];
    const double nrm = sqrt(I.dots[(size_t)idx * 4 + 0]);
    for (uint32_t e = blockIdx.x * BLOCK + threadIdx.x; e < I.nel; e += gridDim.x * BLOCK) {
        T y = G::ld(x, e);
#pragma unroll
        for (int l = 0; l < 2; ++l) y[l] = nrm > 0.0 ? y[l] / nrm : 0.0;
        G::st(x, e, y);
    }
}

// ---------------------------------------------------------------------------
// the k x k tridiagonal matrix: extreme eigenpairs and the padded interval
// ---------------------------------------------------------------------------
// Number of eigenvalues of T below x: negative pivots of the LDL^T
// factorisation of T - x I (Sturm count).
__device__ inline int lz_count_below(const double *al, const double *b2, int m, double x, double pivmin)
{
    int c = 0;
    double q = al[0] - x;
    if (fabs(q) < pivmin) q = -pivmin;
    if (q < 0.0) ++c;
    for (int i = 1; i < m; ++i) {
        q = (al[i] - x) - b2[i - 1] / q;
        if (fabs(q) < pivmin) q = -pivmin;
        if (q < 0.0) ++c;
    }
    return c;
}

// Eigenvalue number `which` (0 = smallest) of T by bisection on the count.
__device__ inline double lz_bisect(const double *al, const double *b2, int m, int which, double lo, double hi,
                                   double pivmin)
{
    for (int it = 0; it < 256; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;   // adjacent doubles
        if (lz_count_below(al, b2, m, mid, pivmin) >= which + 1) hi = mid;
        else lo = mid;
    }
    return 0.5 * (lo + hi);
}

// |last component| of the unit eigenvector of T for the eigenvalue theta:
// two steps of inverse iteration, each a solve with T - theta I factored by
// Gaussian elimination with partial pivoting (tridiagonal form, one extra
// superdiagonal from the row interchanges).  Work arrays of length m in LDS.
__device__ inline double lz_last_component(const double *al, const double *be, int m, double theta, double tnorm,
                                           double *d, double *dl, double *du, double *du2, unsigned char *piv,
                                           double *x)
{
    if (m == 1) return 1.0;
    for (int i = 0; i < m; ++i) {
        d[i] = al[i] - theta;
        du2[i] = 0.0;
        x[i] = 1.0;
    }
    for (int i = 0; i + 1 < m; ++i) {
        dl[i] = be[i];
        du[i] = be[i];
    }
    for (int i = 0; i + 1 < m; ++i) {
        if (fabs(d[i]) >= fabs(dl[i])) {
            piv[i] = 0;
            if (d[i] != 0.0) {
                const double f = dl[i] / d[i];
                dl[i] = f;
                d[i + 1] = d[i + 1] - f * du[i];
            } else {
                dl[i] = 0.0;
            }
        } else {
            piv[i] = 1;
            const double f = d[i] / dl[i];
            d[i] = dl[i];
            dl[i] = f;
            const double tmp = du[i];
            du[i] = d[i + 1];
            d[i + 1] = tmp - f * d[i + 1];
            if (i + 2 < m) {
                du2[i] = du[i + 1];
                du[i + 1] = -f * du[i + 1];
            }
        }
    }
    const double tiny = 2.220446049250313e-16 * (tnorm > 0.0 ? tnorm : 1.0);
    for (int i = 0; i < m; ++i)
        if (d[i] == 0.0) d[i] = tiny;
    for (int pass = 0; pass < 2; ++pass) {
        for (int i = 0; i + 1 < m; ++i) {
            if (!piv[i]) {
                x[i + 1] = x[i + 1] - dl[i] * x[i];
            } else {
                const double tmp = x[i];
                x[i] = x[i + 1];
                x[i + 1] = tmp - dl[i] * x[i];
            }
        }
        x[m - 1] = x[m - 1] / d[m - 1];
        x[m - 2] = (x[m - 2] - du[m - 2] * x[m - 1]) / d[m - 2];
        for (int i = m - 3; i >= 0; --i) x[i] = ((x[i] - du[i] * x[i + 1]) - du2[i] * x[i + 2]) / d[i];
        double s = 0.0;
        for (int i = 0; i < m; ++i) s = fmax(s, fabs(x[i]));
        double n2 = 0.0;
        for (int i = 0; i < m; ++i) {
            x[i] = x[i] / s;
            n2 = n2 + x[i] * x[i];
        }
        const double n = sqrt(n2);
        for (int i = 0; i < m; ++i) x[i] = x[i] / n;
    }
    return fabs(x[m - 1]);
}

// out[0..1]  E_lo, E_hi of H (padded, mapped by E = a lambda + b, clipped)
// out[2..3]  theta_min, theta_max (Ritz values of H~)
// out[4..5]  r_min, r_max (residual bounds, units of H~)
// out[6]     m, the number of Lanczos steps used (a breakdown stops early)
// out[8 + j], out[8 + k + j]  alpha_j, beta_j for j < k
__global__ __launch_bounds__(64) void k_lz_tridiag(const Inst *__restrict__ tab, int32_t k, double pad, double a,
                                                   double b, double clamp_lo, double clamp_hi, double *out)
{
    __shared__ double al[LZ_KMAX], be[LZ_KMAX], b2[LZ_KMAX];
    __shared__ double d[LZ_KMAX], dl[LZ_KMAX], du[LZ_KMAX], du2[LZ_KMAX], x[LZ_KMAX];
    __shared__ unsigned char piv[LZ_KMAX];
    const Inst I = tab[0];
    for (int j = threadIdx.x; j < k; j += blockDim.x) {
        al[j] = I.dots[(size_t)(2 * j + 1) * 4 + 2];
        be[j] = sqrt(I.dots[(size_t)(2 * j + 2) * 4 + 0]);
        b2[j] = be[j] * be[j];
        out[8 + j] = al[j];
        out[8 + k + j] = be[j];
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    int m = k;
    bool stop = false;
    double scale = 0.0;
    for (int j = 0; j < k; ++j) {
        scale = fmax(scale, fmax(fabs(al[j]), be[j]));
        if (be[j] <= LZ_BREAKDOWN * scale) {
            m = j + 1;
            stop = true;
            break;
        }
    }
    // Gershgorin interval of T brackets every eigenvalue
    double glo = al[0], ghi = al[0], tnorm = 0.0;
    for (int i = 0; i < m; ++i) {
        const double r = (i > 0 ? be[i - 1] : 0.0) + (i + 1 < m ? be[i] : 0.0);
        glo = fmin(glo, al[i] - r);
        ghi = fmax(ghi, al[i] + r);
        tnorm = fmax(tnorm, fabs(al[i]) + r);
    }
    const double pivmin = 1e-290 * fmax(1.0, tnorm * tnorm);
    const double margin = 4.440892098500626e-16 * (tnorm > 0.0 ? tnorm : 1.0) + pivmin;
    glo -= margin;
    ghi += margin;
    const double th_lo = lz_bisect(al, b2, m, 0, glo, ghi, pivmin);
    const double th_hi = lz_bisect(al, b2, m, m - 1, glo, ghi, pivmin);
    const double blast = stop ? 0.0 : be[m - 1];
    double r_lo = 0.0, r_hi = 0.0;
    if (blast > 0.0) {
        r_lo = blast * lz_last_component(al, be, m, th_lo, tnorm, d, dl, du, du2, piv, x);
        r_hi = blast * lz_last_component(al, be, m, th_hi, tnorm, d, dl, du, du2, piv, x);
    }
    const double width = th_hi - th_lo;
    const double lo = th_lo - fmax(r_lo, pad * width);
    const double hi = th_hi + fmax(r_hi, pad * width);
    out[0] = fmax(a * lo + b, clamp_lo);
    out[1] = fmin(a * hi + b, clamp_hi);
    out[2] = th_lo;
    out[3] = th_hi;
    out[4] = r_lo;
    out[5] = r_hi;
    out[6] = (double)m;
    out[7] = 0.0;
}

}  // namespace kpm
