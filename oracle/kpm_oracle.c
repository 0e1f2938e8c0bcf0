/*
 * kpm_oracle.c -- plain FP64 CPU oracle for the Kernel Polynomial Method
 * moments (Zhang, Yamagiwa, Okumura, Yunoki, "Performance Acceleration of
 * Kernel Polynomial Method Applying Graphics Processing Units", 2011).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code
 * with the HIP library: it includes no header of it and calls nothing in it.
 *
 * What it computes (Sec. II-A of the paper):
 *   H~   = (H - b) / a                                   Eq. (tilde); b = alpha_+, a = alpha_-
 *   |r_0> = xi_r,  |r_1> = H~|r_0>,  |r_{n+1}> = 2 H~|r_n> - |r_{n-1}>     Eq. (rn)
 *   mu_n = 1/(N R) sum_r Re <r_0|r_n>                     Eq. (munr)  -- "formula A"
 * and, as a second, independent evaluation of the same estimator,
 *   mu_{2n}   = 1/(N R) sum_r ( 2 <r_n|r_n>       - <r_0|r_0> )
 *   mu_{2n+1} = 1/(N R) sum_r ( 2 Re<r_{n+1}|r_n> - Re<r_1|r_0> )       -- "formula B"
 * which follows from T_m T_n = (T_{m+n} + T_{|m-n|})/2 (a consequence of the
 * cosine definition of T_n in Sec. II-A) and the hermiticity of T_n(H~).
 *
 * The random vectors (Sec. II-A, stochastic evaluation of traces) are drawn
 * from the counter-based generator Philox4x64-10 (Salmon, Moraes, Dror, Shaw,
 * SC'11, "Parallel random numbers: as easy as 1, 2, 3"):
 *   key = (seed, 4), counter = (i, floor(r/4), instance, 0), word = r mod 4
 *   Rademacher : xi = +1 if the top bit of the word is 0, else -1
 *   phase      : xi = e^{i phi}, phi = 2 pi k / 2^30 with k = word >> 34, evaluated exactly
 *                reproducibly as the product over the set bits j of k (ascending) of
 *                w_j = e^{2 pi i 2^j / 2^30}; the w_j come from the half-angle recurrence
 *                cos(t/2) = sqrt((1 + cos t)/2), sin(t/2) = sin t / (2 cos(t/2)) started at
 *                e^{i pi/2} = i, e^{i pi} = -1 (IEEE sqrt, division and products only)
 *   unit       : xi_r = e_j with j = (instance + r) mod N
 * so xi depends only on (seed, instance, r, i).  The estimator is normalised
 * by 1/(N R) for the random kinds and by 1/R for unit vectors.
 *
 * Spectral bounds follow the Gershgorin theorem as the paper prescribes
 * (Sec. II-A, below Eq. (tilde)).  As a tighter alternative for the same
 * rescaling step, the Lanczos three-term process (not in the paper; the
 * textbook algorithm, e.g. Golub and Van Loan, Matrix Computations, Sec. 10.1)
 * tridiagonalises H~ from one start vector:
 *   v_0 = xi / ||xi||;  for j = 0, 1, ...:
 *     u = H~ v_j,  alpha_j = Re <v_j|u>,
 *     w = (u - alpha_j v_j) - beta_{j-1} v_{j-1}   (last term absent for j = 0),
 *     beta_j = ||w||,  v_{j+1} = w / beta_j        (v_{j+1} = 0 if beta_j = 0)
 * with the same matrix-vector product and double-double dot products as the
 * recursion (each dot rounded once to FP64).
 *
 * Arithmetic conventions (all FP64, compiled with -ffp-contract=off so that
 * nothing is fused):
 *   d_i  = (eps_i - b) / a
 *   real hopping      H~_ij = (-t) / a
 *   spin hopping      z = u_i^dag u_j = c_i c_j + (x_i x_j + y_i y_j) + i (x_i y_j - y_i x_j),
 *                     H~_ij = ((-t) z_re / a, (-t) z_im / a),
 *                     u_i = (c_i, x_i + i y_i) = (cos(theta_i/2), e^{i phi_i} sin(theta_i/2))
 *   matrix-vector     acc = d_i v_i; then acc += H~_ij v_j over the neighbour
 *                     slots in the order -x, +x, -y, +y, -z, +z (periodic);
 *                     complex products as (hr vr - hi vi, hr vi + hi vr)
 *   recursion         r_1 = acc;  r_{n+1} = 2 acc - r_{n-1}
 *   dot products      exact products (two_prod with fma) accumulated as a
 *                     double-double (Ogita, Rump, Oishi, "Accurate sum and dot
 *                     product", SIAM J. Sci. Comput. 26, 2005), over fixed
 *                     site chunks, chunks then vectors in ascending order;
 *                     the moments are formed and normalised in double-double
 *                     and rounded once.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define KPMO_OK 0
#define KPMO_ERR_ARG 1
#define KPMO_ERR_MEM 2

enum { VEC_RADEMACHER = 0, VEC_PHASE = 1, VEC_UNIT = 2 };
enum { HOP_REAL = 0, HOP_SPIN = 1 };

/* ------------------------------------------------------------------------ */
/* Philox4x64-10                                                             */
/* ------------------------------------------------------------------------ */
static const uint64_t PHILOX_M0 = 0xD2E7470EE14C6C93ULL;
static const uint64_t PHILOX_M1 = 0xCA5A826395121157ULL;
static const uint64_t PHILOX_W0 = 0x9E3779B97F4A7C15ULL; /* golden ratio */
static const uint64_t PHILOX_W1 = 0xBB67AE8584CAA73BULL; /* sqrt(3) - 1  */

void kpmo_philox4x64_10(const uint64_t ctr_in[4], const uint64_t key_in[2], uint64_t out[4])
{
    uint64_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint64_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { k0 += PHILOX_W0; k1 += PHILOX_W1; }
        unsigned __int128 p0 = (unsigned __int128)PHILOX_M0 * c0;
        unsigned __int128 p1 = (unsigned __int128)PHILOX_M1 * c2;
        uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        c0 = hi1 ^ c1 ^ k0;
        c1 = lo1;
        c2 = hi0 ^ c3 ^ k1;
        c3 = lo0;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* w_j = e^{2 pi i 2^j / 2^30}, j = 0..29 (see the header comment). */
#define PHASE_BITS 30
static double phase_w[PHASE_BITS][2];
static int phase_ready = 0;
static void phase_table(void)
{
    if (phase_ready) return;
    /* angle 2 pi / 2^m for m = 1 (pi), 2 (pi/2), ..., 30; w_j has m = 30 - j */
    double c = -1.0, sn = 0.0;                 /* m = 1 */
    phase_w[PHASE_BITS - 1][0] = c;
    phase_w[PHASE_BITS - 1][1] = sn;
    c = 0.0; sn = 1.0;                          /* m = 2 */
    phase_w[PHASE_BITS - 2][0] = c;
    phase_w[PHASE_BITS - 2][1] = sn;
    for (int m = 3; m <= PHASE_BITS; ++m) {
        double ch = sqrt((1.0 + c) / 2.0);
        double sh = sn / (2.0 * ch);
        c = ch;
        sn = sh;
        phase_w[PHASE_BITS - m][0] = c;
        phase_w[PHASE_BITS - m][1] = sn;
    }
    phase_ready = 1;
}

/* Entry xi_{r,i} of the start vector, as (re, im). */
static void start_entry(int vec_kind, uint64_t seed, uint64_t instance,
                        int64_t N, int64_t r, int64_t i, double *re, double *im)
{
    if (vec_kind == VEC_UNIT) {
        int64_t j = (int64_t)((instance + (uint64_t)r) % (uint64_t)N);
        *re = (i == j) ? 1.0 : 0.0;
        *im = 0.0;
        return;
    }
    uint64_t ctr[4] = { (uint64_t)i, (uint64_t)(r / 4), instance, 0 };
    uint64_t key[2] = { seed, 4 };
    uint64_t w[4];
    kpmo_philox4x64_10(ctr, key, w);
    uint64_t word = w[r % 4];
    if (vec_kind == VEC_RADEMACHER) {
        *re = (word >> 63) ? -1.0 : 1.0;
        *im = 0.0;
    } else {
        uint64_t k = word >> (64 - PHASE_BITS);
        double zr = 1.0, zi = 0.0;
        int started = 0;
        for (int j = 0; j < PHASE_BITS; ++j) {
            if (!((k >> j) & 1)) continue;
            double wr = phase_w[j][0], wi = phase_w[j][1];
            if (!started) {
                zr = wr; zi = wi; started = 1;
            } else {
                double tr = zr * wr - zi * wi;
                double ti = zr * wi + zi * wr;
                zr = tr; zi = ti;
            }
        }
        *re = zr;
        *im = zi;
    }
}

void kpmo_start_vectors(int vec_kind, uint64_t seed, uint64_t instance, int64_t N, int R,
                        double *re /* [R][N] */, double *im /* [R][N] */)
{
    phase_table();
    for (int64_t r = 0; r < R; ++r)
        for (int64_t i = 0; i < N; ++i)
            start_entry(vec_kind, seed, instance, N, r, i, &re[r * N + i], &im[r * N + i]);
}

/* ------------------------------------------------------------------------ */
/* double-double helpers (error-free transformations)                        */
/* ------------------------------------------------------------------------ */
typedef struct { double hi, lo; } dd;

static inline dd two_sum(double a, double b)
{
    double s = a + b;
    double bb = s - a;
    double e = (a - (s - bb)) + (b - bb);
    dd r = { s, e };
    return r;
}
static inline dd quick_two_sum(double a, double b)
{
    double s = a + b;
    double e = b - (s - a);
    dd r = { s, e };
    return r;
}
static inline dd dd_add(dd x, dd y)
{
    dd s = two_sum(x.hi, y.hi);
    dd t = two_sum(x.lo, y.lo);
    s.lo += t.hi;
    s = quick_two_sum(s.hi, s.lo);
    s.lo += t.lo;
    return quick_two_sum(s.hi, s.lo);
}
/* accumulate the exact product x*y into acc */
static inline dd dd_fma_acc(dd acc, double x, double y)
{
    double p = x * y;
    double pe = fma(x, y, -p);
    dd s = two_sum(acc.hi, p);
    s.lo += acc.lo + pe;
    return quick_two_sum(s.hi, s.lo);
}
static inline dd dd_scale2(dd x) { dd r = { 2.0 * x.hi, 2.0 * x.lo }; return r; }
static inline dd dd_neg(dd x) { dd r = { -x.hi, -x.lo }; return r; }
static inline dd dd_div_d(dd x, double b)
{
    double q1 = x.hi / b;
    double p = q1 * b;
    double pe = fma(q1, b, -p);
    double rem = ((x.hi - p) - pe) + x.lo;
    double q2 = rem / b;
    return quick_two_sum(q1, q2);
}

/* ------------------------------------------------------------------------ */
/* operator: H~ in neighbour-slot form                                       */
/* ------------------------------------------------------------------------ */
typedef struct {
    int64_t N;
    int nslot;           /* neighbour slots per site (lattice) */
    int64_t *nbr;        /* [N][nslot] (lattice) */
    double *hre, *him;   /* [N][nslot] (lattice) or [nnz] (CSR off-diagonal, 0 on diagonal entries) */
    double *diag;        /* [N] */
    const int64_t *row_ptr; const int32_t *col;  /* CSR */
    int is_csr;
} oper;

static void oper_free(oper *op)
{
    free(op->nbr); free(op->hre); free(op->him); free(op->diag);
    memset(op, 0, sizeof(*op));
}

/* periodic neighbour of site i along axis ax with step dir (-1 or +1) */
static int64_t lattice_neighbour(const int64_t L[3], int64_t i, int ax, int dir)
{
    int64_t x = i % L[0];
    int64_t y = (i / L[0]) % L[1];
    int64_t z = i / (L[0] * L[1]);
    int64_t c[3] = { x, y, z };
    c[ax] = (c[ax] + dir + L[ax]) % L[ax];
    return c[0] + L[0] * (c[1] + L[1] * c[2]);
}

/* z = u_i^dag u_j for spinors given as (c, x, y) triples */
static void spin_overlap(const double *sp, int64_t i, int64_t j, double *zr, double *zi)
{
    double ci = sp[3 * i], xi = sp[3 * i + 1], yi = sp[3 * i + 2];
    double cj = sp[3 * j], xj = sp[3 * j + 1], yj = sp[3 * j + 2];
    *zr = ci * cj + (xi * xj + yi * yj);
    *zi = xi * yj - yi * xj;
}

static int build_lattice_oper(oper *op, int dim, const int64_t L[3], double t, int hop,
                              const double *onsite, const double *spinor, double a, double b)
{
    int64_t LL[3] = { L[0], L[1], dim == 3 ? L[2] : 1 };
    op->N = LL[0] * LL[1] * LL[2];
    op->nslot = 2 * dim;
    op->is_csr = 0;
    int64_t N = op->N;
    int ns = op->nslot;
    op->nbr = (int64_t *)malloc(sizeof(int64_t) * N * ns);
    op->hre = (double *)malloc(sizeof(double) * N * ns);
    op->him = (double *)malloc(sizeof(double) * N * ns);
    op->diag = (double *)malloc(sizeof(double) * N);
    if (!op->nbr || !op->hre || !op->him || !op->diag) { oper_free(op); return KPMO_ERR_MEM; }
    for (int64_t i = 0; i < N; ++i) {
        double eps = onsite ? onsite[i] : 0.0;
        op->diag[i] = (eps - b) / a;
        for (int s = 0; s < ns; ++s) {
            int ax = s / 2, dir = (s % 2) ? +1 : -1;
            int64_t j = lattice_neighbour(LL, i, ax, dir);
            op->nbr[i * ns + s] = j;
            if (hop == HOP_REAL) {
                op->hre[i * ns + s] = (-t) / a;
                op->him[i * ns + s] = 0.0;
            } else {
                double zr, zi;
                spin_overlap(spinor, i, j, &zr, &zi);
                op->hre[i * ns + s] = ((-t) * zr) / a;
                op->him[i * ns + s] = ((-t) * zi) / a;
            }
        }
    }
    return KPMO_OK;
}

static int build_csr_oper(oper *op, int64_t N, const int64_t *row_ptr, const int32_t *col,
                          const double *val_re, const double *val_im, double a, double b)
{
    int64_t nnz = row_ptr[N];
    op->N = N;
    op->is_csr = 1;
    op->nslot = 0;
    op->row_ptr = row_ptr;
    op->col = col;
    op->hre = (double *)malloc(sizeof(double) * (nnz > 0 ? nnz : 1));
    op->him = (double *)malloc(sizeof(double) * (nnz > 0 ? nnz : 1));
    op->diag = (double *)malloc(sizeof(double) * (N > 0 ? N : 1));
    if (!op->hre || !op->him || !op->diag) { oper_free(op); return KPMO_ERR_MEM; }
    for (int64_t i = 0; i < N; ++i) {
        double hii = 0.0;
        for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
            if (col[k] == i) {
                hii = hii + val_re[k];
                op->hre[k] = 0.0;
                op->him[k] = 0.0;
            } else {
                op->hre[k] = val_re[k] / a;
                op->him[k] = val_im ? val_im[k] / a : 0.0;
            }
        }
        op->diag[i] = (hii - b) / a;
    }
    return KPMO_OK;
}

/* out = 2 H~ v - prev (or H~ v when prev is NULL); vectors as split re/im */
static void apply_step(const oper *op, const double *vr, const double *vi,
                       const double *pr, const double *pi, double *outr, double *outi)
{
    int64_t N = op->N;
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) {
        double ar = op->diag[i] * vr[i];
        double ai = op->diag[i] * vi[i];
        if (!op->is_csr) {
            int ns = op->nslot;
            for (int s = 0; s < ns; ++s) {
                int64_t j = op->nbr[i * ns + s];
                double hr = op->hre[i * ns + s], hi = op->him[i * ns + s];
                ar = ar + (hr * vr[j] - hi * vi[j]);
                ai = ai + (hr * vi[j] + hi * vr[j]);
            }
        } else {
            for (int64_t k = op->row_ptr[i]; k < op->row_ptr[i + 1]; ++k) {
                int64_t j = op->col[k];
                if (j == i) continue;
                double hr = op->hre[k], hi = op->him[k];
                ar = ar + (hr * vr[j] - hi * vi[j]);
                ai = ai + (hr * vi[j] + hi * vr[j]);
            }
        }
        if (pr) {
            outr[i] = 2.0 * ar - pr[i];
            outi[i] = 2.0 * ai - pi[i];
        } else {
            outr[i] = ar;
            outi[i] = ai;
        }
    }
}

/* Re <a|b> as a double-double; the sites are split into a fixed number of
 * chunks (independent of the thread count), each summed in order, and the
 * chunk results are added in order, so the result is reproducible. */
#define DOT_CHUNKS 64
static dd dot_re(int64_t N, const double *ar, const double *ai, const double *br, const double *bi)
{
    dd part[DOT_CHUNKS];
    #pragma omp parallel for schedule(static)
    for (int c = 0; c < DOT_CHUNKS; ++c) {
        int64_t lo = N * c / DOT_CHUNKS, hi = N * (c + 1) / DOT_CHUNKS;
        dd s = { 0.0, 0.0 };
        for (int64_t i = lo; i < hi; ++i) {
            s = dd_fma_acc(s, ar[i], br[i]);
            s = dd_fma_acc(s, ai[i], bi[i]);
        }
        part[c] = s;
    }
    dd s = { 0.0, 0.0 };
    for (int c = 0; c < DOT_CHUNKS; ++c) s = dd_add(s, part[c]);
    return s;
}

/*
 * Core: run the recursion for each vector r in turn (the paper's view: every
 * random vector is an independent recursion, Sec. III-A) and accumulate
 *   S_nn[n] = sum_r <r_n|r_n>,   S_nm[n] = sum_r Re<r_n|r_{n-1}>  (n >= 1),
 *   S_0n[n] = sum_r Re<r_0|r_n>
 * in double-double.  nvec = ceil(M/2)+... vectors r_0..r_K, K = floor(M/2),
 * are needed for formula B; formula A needs r_0..r_{M-1}.
 */
static int run_moments(const oper *op, int M, int R, int vec_kind, uint64_t seed,
                       uint64_t instance, double *mu_B, double *mu_A,
                       double *dots_out /* optional [K+1][2][2]: (nn, nm) as (hi, lo) */)
{
    int64_t N = op->N;
    if (M < 1 || R < 1 || N < 1) return KPMO_ERR_ARG;
    int K = M / 2;                       /* highest vector index formula B needs */
    phase_table();
    int nmax = mu_A ? (M - 1 > K ? M - 1 : K) : K;
    dd *Snn = (dd *)calloc((size_t)nmax + 2, sizeof(dd));
    dd *Snm = (dd *)calloc((size_t)nmax + 2, sizeof(dd));
    dd *S0n = (dd *)calloc((size_t)nmax + 2, sizeof(dd));
    double *buf = (double *)malloc(sizeof(double) * (size_t)N * 8);
    if (!Snn || !Snm || !S0n || !buf) {
        free(Snn); free(Snm); free(S0n); free(buf);
        return KPMO_ERR_MEM;
    }
    double *r0r = buf, *r0i = buf + N;
    double *ar = buf + 2 * N, *ai = buf + 3 * N;   /* r_{n-1} */
    double *br = buf + 4 * N, *bi = buf + 5 * N;   /* r_n     */
    double *cr = buf + 6 * N, *ci = buf + 7 * N;   /* r_{n+1} */

    for (int r = 0; r < R; ++r) {
        #pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < N; ++i)
            start_entry(vec_kind, seed, instance, N, r, i, &r0r[i], &r0i[i]);
        /* n = 0 */
        Snn[0] = dd_add(Snn[0], dot_re(N, r0r, r0i, r0r, r0i));
        S0n[0] = dd_add(S0n[0], dot_re(N, r0r, r0i, r0r, r0i));
        if (nmax >= 1) {
            apply_step(op, r0r, r0i, NULL, NULL, br, bi);       /* r_1 = H~ r_0 */
            Snn[1] = dd_add(Snn[1], dot_re(N, br, bi, br, bi));
            Snm[1] = dd_add(Snm[1], dot_re(N, br, bi, r0r, r0i));
            S0n[1] = dd_add(S0n[1], dot_re(N, r0r, r0i, br, bi));
            memcpy(ar, r0r, sizeof(double) * N);
            memcpy(ai, r0i, sizeof(double) * N);
        }
        for (int n = 1; n < nmax; ++n) {
            apply_step(op, br, bi, ar, ai, cr, ci);             /* r_{n+1} = 2 H~ r_n - r_{n-1} */
            Snn[n + 1] = dd_add(Snn[n + 1], dot_re(N, cr, ci, cr, ci));
            Snm[n + 1] = dd_add(Snm[n + 1], dot_re(N, cr, ci, br, bi));
            S0n[n + 1] = dd_add(S0n[n + 1], dot_re(N, r0r, r0i, cr, ci));
            double *tr = ar, *ti = ai;
            ar = br; ai = bi; br = cr; bi = ci; cr = tr; ci = ti;
        }
    }

    /* Normalisation of the trace estimator: random entries have unit variance, so
     * <r|r> ~ N and the factor is 1/(N R); unit vectors have <r|r> = 1 and the
     * factor is 1/R (with R = N this is the exact trace of Eq. (DoStr)). */
    double NR = (vec_kind == VEC_UNIT) ? (double)R : (double)N * (double)R;
    /* formula B */
    for (int m = 0; m < M; ++m) {
        dd v;
        if (m == 0) v = Snn[0];
        else if (m == 1) v = Snm[1];
        else if (m % 2 == 0) v = dd_add(dd_scale2(Snn[m / 2]), dd_neg(Snn[0]));
        else v = dd_add(dd_scale2(Snm[m / 2 + 1]), dd_neg(Snm[1]));
        dd q = dd_div_d(v, NR);
        mu_B[m] = q.hi + q.lo;
    }
    /* formula A (the paper's direct estimator, Eq. (munr)) */
    if (mu_A) {
        for (int m = 0; m < M; ++m) {
            dd q = dd_div_d(S0n[m], NR);
            mu_A[m] = q.hi + q.lo;
        }
    }
    if (dots_out) {
        for (int n = 0; n <= K; ++n) {
            dots_out[4 * n + 0] = Snn[n].hi;
            dots_out[4 * n + 1] = Snn[n].lo;
            dots_out[4 * n + 2] = Snm[n].hi;
            dots_out[4 * n + 3] = Snm[n].lo;
        }
    }
    free(Snn); free(Snm); free(S0n); free(buf);
    return KPMO_OK;
}

/* Lanczos coefficients alpha[0..k), beta[0..k) of H~ from start vector r = 0
 * of kind vec_kind (see the header comment). */
static int run_lanczos(const oper *op, int k, int vec_kind, uint64_t seed, uint64_t instance,
                       double *alpha, double *beta)
{
    int64_t N = op->N;
    if (k < 1 || N < 1) return KPMO_ERR_ARG;
    phase_table();
    double *buf = (double *)malloc(sizeof(double) * (size_t)N * 6);
    if (!buf) return KPMO_ERR_MEM;
    double *pr = buf, *pi = buf + N;            /* v_{j-1} */
    double *vr = buf + 2 * N, *vi = buf + 3 * N;  /* v_j */
    double *ur = buf + 4 * N, *ui = buf + 5 * N;  /* H~ v_j, then w */
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) {
        start_entry(vec_kind, seed, instance, N, 0, i, &vr[i], &vi[i]);
        pr[i] = 0.0;
        pi[i] = 0.0;
    }
    dd n0 = dot_re(N, vr, vi, vr, vi);
    double nrm = sqrt(n0.hi + n0.lo);
    for (int64_t i = 0; i < N; ++i) {
        vr[i] = vr[i] / nrm;
        vi[i] = vi[i] / nrm;
    }
    double beta_prev = 0.0;
    for (int j = 0; j < k; ++j) {
        apply_step(op, vr, vi, NULL, NULL, ur, ui);            /* u = H~ v_j */
        dd a = dot_re(N, vr, vi, ur, ui);
        double al = a.hi + a.lo;
        #pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < N; ++i) {
            double wr = ur[i] - al * vr[i];
            double wi = ui[i] - al * vi[i];
            if (j > 0) {
                wr = wr - beta_prev * pr[i];
                wi = wi - beta_prev * pi[i];
            }
            ur[i] = wr;
            ui[i] = wi;
        }
        dd b2 = dot_re(N, ur, ui, ur, ui);
        double be = sqrt(b2.hi + b2.lo);
        alpha[j] = al;
        beta[j] = be;
        /* v_{j-1} <- v_j, v_j <- w / beta_j */
        #pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < N; ++i) {
            pr[i] = vr[i];
            pi[i] = vi[i];
            vr[i] = be > 0.0 ? ur[i] / be : 0.0;
            vi[i] = be > 0.0 ? ui[i] / be : 0.0;
        }
        beta_prev = be;
    }
    free(buf);
    return KPMO_OK;
}

static void set_threads(int nthreads)
{
    if (nthreads > 0) omp_set_num_threads(nthreads);
}

int kpmo_max_threads(void) { return omp_get_max_threads(); }

/* ------------------------------------------------------------------------ */
/* public entry points (host pointers throughout)                            */
/* ------------------------------------------------------------------------ */

/* dim: 2 or 3; L: extents (L[2] ignored for dim 2); hop: 0 real, 1 spin;
 * onsite: N values or NULL; spinor: N*3 values (c, x, y) when hop == 1. */
int kpmo_moments_lattice(int dim, const int64_t *L, double t, int hop,
                         const double *onsite, const double *spinor,
                         double a, double b, int M, int R, int vec_kind,
                         uint64_t seed, uint64_t instance, int nthreads,
                         double *mu_B, double *mu_A, double *dots_out)
{
    if ((dim != 2 && dim != 3) || !(a > 0.0) || M < 1 || R < 1) return KPMO_ERR_ARG;
    if (hop == HOP_SPIN && !spinor) return KPMO_ERR_ARG;
    for (int d = 0; d < dim; ++d) if (L[d] < 1) return KPMO_ERR_ARG;
    set_threads(nthreads);
    oper op;
    memset(&op, 0, sizeof(op));
    int st = build_lattice_oper(&op, dim, L, t, hop, onsite, spinor, a, b);
    if (st) return st;
    st = run_moments(&op, M, R, vec_kind, seed, instance, mu_B, mu_A, dots_out);
    oper_free(&op);
    return st;
}

int kpmo_moments_csr(int64_t N, const int64_t *row_ptr, const int32_t *col,
                     const double *val_re, const double *val_im,
                     double a, double b, int M, int R, int vec_kind,
                     uint64_t seed, uint64_t instance, int nthreads,
                     double *mu_B, double *mu_A, double *dots_out)
{
    if (N < 1 || !(a > 0.0) || M < 1 || R < 1) return KPMO_ERR_ARG;
    set_threads(nthreads);
    oper op;
    memset(&op, 0, sizeof(op));
    int st = build_csr_oper(&op, N, row_ptr, col, val_re, val_im, a, b);
    if (st) return st;
    st = run_moments(&op, M, R, vec_kind, seed, instance, mu_B, mu_A, dots_out);
    op.row_ptr = NULL; op.col = NULL;
    oper_free(&op);
    return st;
}

/* Gershgorin discs (Sec. II-A): E_lo = min_i (Re H_ii - sum_{j != i} |H_ij|),
 * E_hi = max_i (Re H_ii + sum_{j != i} |H_ij|); lattice neighbour slots count
 * as off-diagonal entries even when a slot wraps onto the site itself. */
int kpmo_gershgorin_lattice(int dim, const int64_t *L, double t, int hop,
                            const double *onsite, const double *spinor,
                            double *e_lo, double *e_hi)
{
    if (dim != 2 && dim != 3) return KPMO_ERR_ARG;
    int64_t LL[3] = { L[0], L[1], dim == 3 ? L[2] : 1 };
    int64_t N = LL[0] * LL[1] * LL[2];
    double lo = INFINITY, hi = -INFINITY;
    for (int64_t i = 0; i < N; ++i) {
        double rad = 0.0;
        for (int s = 0; s < 2 * dim; ++s) {
            int64_t j = lattice_neighbour(LL, i, s / 2, (s % 2) ? +1 : -1);
            if (hop == HOP_REAL) {
                rad = rad + fabs(t);
            } else {
                double zr, zi;
                spin_overlap(spinor, i, j, &zr, &zi);
                rad = rad + hypot((-t) * zr, (-t) * zi);
            }
        }
        double eps = onsite ? onsite[i] : 0.0;
        if (eps - rad < lo) lo = eps - rad;
        if (eps + rad > hi) hi = eps + rad;
    }
    *e_lo = lo;
    *e_hi = hi;
    return KPMO_OK;
}

int kpmo_gershgorin_csr(int64_t N, const int64_t *row_ptr, const int32_t *col,
                        const double *val_re, const double *val_im,
                        double *e_lo, double *e_hi)
{
    double lo = INFINITY, hi = -INFINITY;
    for (int64_t i = 0; i < N; ++i) {
        double hii = 0.0, rad = 0.0;
        for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
            if (col[k] == i) hii = hii + val_re[k];
            else rad = rad + hypot(val_re[k], val_im ? val_im[k] : 0.0);
        }
        if (hii - rad < lo) lo = hii - rad;
        if (hii + rad > hi) hi = hii + rad;
    }
    *e_lo = lo;
    *e_hi = hi;
    return KPMO_OK;
}

/* Lanczos coefficients of H~ = (H - b)/a (see the header comment). */
int kpmo_lanczos_lattice(int dim, const int64_t *L, double t, int hop,
                         const double *onsite, const double *spinor,
                         double a, double b, int k, int vec_kind,
                         uint64_t seed, uint64_t instance, int nthreads,
                         double *alpha, double *beta)
{
    if ((dim != 2 && dim != 3) || !(a > 0.0) || k < 1 || !alpha || !beta) return KPMO_ERR_ARG;
    if (hop == HOP_SPIN && !spinor) return KPMO_ERR_ARG;
    for (int d = 0; d < dim; ++d) if (L[d] < 1) return KPMO_ERR_ARG;
    set_threads(nthreads);
    oper op;
    memset(&op, 0, sizeof(op));
    int st = build_lattice_oper(&op, dim, L, t, hop, onsite, spinor, a, b);
    if (st) return st;
    st = run_lanczos(&op, k, vec_kind, seed, instance, alpha, beta);
    oper_free(&op);
    return st;
}

int kpmo_lanczos_csr(int64_t N, const int64_t *row_ptr, const int32_t *col,
                     const double *val_re, const double *val_im,
                     double a, double b, int k, int vec_kind,
                     uint64_t seed, uint64_t instance, int nthreads,
                     double *alpha, double *beta)
{
    if (N < 1 || !(a > 0.0) || k < 1 || !alpha || !beta) return KPMO_ERR_ARG;
    set_threads(nthreads);
    oper op;
    memset(&op, 0, sizeof(op));
    int st = build_csr_oper(&op, N, row_ptr, col, val_re, val_im, a, b);
    if (st) return st;
    st = run_lanczos(&op, k, vec_kind, seed, instance, alpha, beta);
    op.row_ptr = NULL; op.col = NULL;
    oper_free(&op);
    return st;
}
