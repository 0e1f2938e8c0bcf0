/*
 * kpm.h -- C ABI of libkpm, the MI355X (gfx950) implementation of the hot
 * path of the Kernel Polynomial Method (KPM): the Chebyshev vector recursion
 * over R random vectors on a rescaled sparse tight-binding Hamiltonian, fused
 * with the moment dot products, plus the Jackson-damped density of states.
 *
 * The method follows Zhang, Yamagiwa, Okumura, Yunoki, "Performance
 * Acceleration of Kernel Polynomial Method Applying Graphics Processing
 * Units" (2011), Sec. II-A and Sec. III:
 *   H~ = (H - b) / a                       Eq. (tilde), a = alpha_-, b = alpha_+
 *   |r_0> = xi, |r_1> = H~|r_0>, |r_{n+1}> = 2 H~|r_n> - |r_{n-1}>   Eq. (rn)
 *   mu_n = 1/(N R) sum_r <r_0|r_n>          Eq. (munr), evaluated through
 *   mu_{2n} = 2<r_n|r_n>/(N R) - mu_0,  mu_{2n+1} = 2 Re<r_{n+1}|r_n>/(N R) - mu_1
 *   f(x) = [g_0 mu_0 + 2 sum g_n mu_n T_n(x)] / (pi sqrt(1-x^2))     Eq. (fKPM)
 *
 * Conventions for every entry point:
 *  - Pointers named *_dev are device pointers (HBM of the current HIP device);
 *    all other pointers are host pointers.  The caller owns every array it
 *    passes.  Device arrays must stay valid until the work enqueued on the
 *    given stream has completed.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *    Work is enqueued asynchronously; outputs in device memory are valid once
 *    the stream has reached that point.
 *  - Every call returns a kpm_status and never aborts.  On an argument error
 *    nothing is enqueued and outputs are left untouched.  KPM_ERR_DEVICE
 *    reports a HIP runtime error seen while enqueuing.
 *  - A kpm_ham or kpm_solve handle must not be used from two host threads at
 *    the same time.  Two solves may run concurrently on different streams if
 *    each has its own workspace.
 */
#ifndef KPM_H
#define KPM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    KPM_OK = 0,
    KPM_ERR_INVALID_ARG = 1,   /* a size, pointer or enum is out of range          */
    KPM_ERR_OUT_OF_MEMORY = 2, /* a device allocation failed                       */
    KPM_ERR_DEVICE = 3,        /* a HIP call failed                                */
    KPM_ERR_BOUNDS = 4,        /* scaled spectrum may leave [-1, 1], or divergence */
    KPM_ERR_UNSUPPORTED = 5,   /* a size beyond what the kernels index             */
    KPM_ERR_WORKSPACE = 6      /* workspace missing, misaligned or too small       */
} kpm_status;

/* Operator kinds.  Lattices are periodic; site i = x + Lx (y + Ly z). */
typedef enum { KPM_SQUARE_2D = 2, KPM_CUBIC_3D = 3, KPM_CSR = 10 } kpm_kind;

/* Lattice hopping.  REAL: H_ij = -t on every nearest-neighbour bond.
 * SPIN: H_ij = -t u_i^dag u_j with u_i = (cos(theta_i/2), e^{i phi_i} sin(theta_i/2)),
 * i.e. -t [cos(th_i/2) cos(th_j/2) + sin(th_i/2) sin(th_j/2) e^{-i(phi_i - phi_j)}]. */
typedef enum { KPM_HOP_REAL = 0, KPM_HOP_SPIN = 1 } kpm_hop;

/* Precision of the vector recursion.  Moments are always accumulated in FP64. */
typedef enum { KPM_F64 = 0, KPM_F32 = 1 } kpm_prec;

/* Start vectors (Sec. II-A, stochastic evaluation of traces), drawn on the
 * device from Philox4x64-10 (Salmon et al., SC'11) with key (seed, 4) and
 * counter (i, floor(r/4), instance, 0), word r mod 4:
 *   RADEMACHER: xi_{r,i} = +1 or -1 (top bit of the word);   normalisation 1/(N R)
 *   PHASE:      xi_{r,i} = e^{i phi}, phi = 2 pi k / 2^30, k = word >> 34; e^{i phi} is the
 *               ordered product over the set bits j of k (ascending) of w_j = e^{2 pi i 2^j/2^30},
 *               w_j from the half-angle recurrence cos(t/2) = sqrt((1+cos t)/2),
 *               sin(t/2) = sin t/(2 cos(t/2)) started at e^{i pi} and e^{i pi/2} (IEEE
 *               operations only, so reproducible bit for bit);            normalisation 1/(N R)
 *   UNIT:       xi_r = e_j, j = (instance + r) mod N;        normalisation 1/R
 * With UNIT and R = N the moments are the exact traces Tr T_n(H~)/N (Eq. (DoStr)). */
typedef enum { KPM_VEC_RADEMACHER = 0, KPM_VEC_PHASE = 1, KPM_VEC_UNIT = 2 } kpm_vec;

/* Hamiltonian description (Sec. II-A; the paper's lattice of Sec. IV-A is a
 * KPM_CUBIC_3D with t = 1 and no on-site term).  All arrays are device arrays
 * of FP64 values (indices as stated).
 *   kind, L[0..2] (L[2] ignored for 2D), t, hop: lattice geometry and hopping;
 *   onsite_dev: N on-site energies H_ii, or NULL for zero;
 *   spinor_dev: N x 3 values (cos(th/2), sin(th/2) cos(phi), sin(th/2) sin(phi))
 *               per site, required when hop == KPM_HOP_SPIN;
 *   CSR (kind == KPM_CSR): n rows, row_ptr_dev[n+1] (int64), col_dev[nnz] (int32),
 *               val_re_dev[nnz], val_im_dev[nnz] or NULL for a real matrix.
 *               Entries with equal (row, col) are summed.  H must be Hermitian. */
typedef struct {
    int32_t kind;
    int32_t hop;
    int64_t L[3];
    double t;
    const double *onsite_dev;
    const double *spinor_dev;
    int64_t n;
    int64_t nnz;
    const int64_t *row_ptr_dev;
    const int32_t *col_dev;
    const double *val_re_dev;
    const double *val_im_dev;
} kpm_ham_desc;

typedef struct kpm_ham kpm_ham;     /* opaque: the scaled operator in device memory */
typedef struct kpm_solve kpm_solve; /* opaque: one solve whose state lives in a workspace */

/* Human-readable name of a status code (static string; never NULL, "unknown
 * status" for a value outside kpm_status).  A diagnostic of this library, not an
 * operation of the method. */
const char *kpm_status_string(kpm_status st);

/* Name of the last HIP runtime error a call of this thread ran into (behind
 * KPM_ERR_DEVICE and allocation failures); "no error" if none. */
const char *kpm_last_hip_error(void);

/* Gershgorin bounds of H (Sec. II-A, below Eq. (tilde)):
 *   E_lo = min_i (Re H_ii - sum_{j!=i} |H_ij|),  E_hi = max_i (Re H_ii + sum_{j!=i} |H_ij|),
 * computed in FP64 on the device.  A lattice neighbour slot that wraps onto the
 * site itself (extent 1 or 2) counts as an off-diagonal entry.
 * bounds_dev: device array of 2 doubles receiving (E_lo, E_hi). */
kpm_status kpm_bounds_gershgorin(const kpm_ham_desc *desc, double *bounds_dev, void *stream);

/* Lanczos estimate of the spectral interval (an alternative to Gershgorin for
 * the rescaling of Eq. (tilde); the process itself is the textbook three-term
 * recurrence, not part of the paper).  h must be an FP64 operator (any a, b;
 * a = 1, b = 0 gives H itself).  From one start vector (random phases for a
 * complex operator, +-1 otherwise; Philox key (seed, 4), vector 0, instance 0)
 * it runs k steps
 *   v_0 = xi/||xi||;  u = H~ v_j,  alpha_j = Re<v_j|u>,
 *   w = (u - alpha_j v_j) - beta_{j-1} v_{j-1},  beta_j = ||w||,  v_{j+1} = w/beta_j
 * with double-double dot products, then on the device takes the extreme
 * eigenvalues theta of the tridiagonal matrix T_m (m = k, or fewer when some
 * beta_j <= 1e-12 max(|alpha_i|, beta_i; i <= j), an invariant subspace), their
 * residual bounds r = beta_{m-1} |y_{m-1}| (0 after such a breakdown), and
 *   [theta_min - max(r_min, pad w), theta_max + max(r_max, pad w)],  w = theta_max - theta_min,
 * mapped to H by E = a lambda + b and clipped to [clamp_lo, clamp_hi] (pass an
 * interval known to enclose the spectrum, such as Gershgorin's, or +-inf).
 * Ritz values lie inside the spectrum and approach its ends from inside, so
 * the padding is what makes the interval enclose it; a too small interval shows
 * up as moments above 1 in modulus.
 * out_dev: device array of 8 + 2k doubles:
 *   [0] E_lo, [1] E_hi, [2] theta_min, [3] theta_max, [4] r_min, [5] r_max
 *   (these four in units of H~), [6] m, [7] 0, [8 + j] alpha_j, [8 + k + j] beta_j.
 * 1 <= k <= 512, pad >= 0.  workspace_dev: kpm_lanczos_workspace_bytes(h, k)
 * bytes, 256-byte aligned.  KPM_ERR_UNSUPPORTED for an FP32 operator. */
size_t kpm_lanczos_workspace_bytes(const kpm_ham *h, int32_t k);
kpm_status kpm_bounds_lanczos(kpm_ham *h, int32_t k, uint64_t seed, double pad, double clamp_lo,
                              double clamp_hi, void *workspace_dev, size_t ws_bytes, double *out_dev,
                              void *stream);

/* The dense-H variant of the recursion (the paper's own kernel design, Sec. III;
 * its H_SIZE experiments of Sec. IV): H is a dense real symmetric D x D matrix
 * (H_dev, row-major FP64, device memory), H~ = (H - b)/a is formed in the
 * workspace ((H_ii - b)/a on the diagonal, H_ij/a off it), and each of the
 * floor(M/2) steps computes V_{n+1} = 2 H~ V_n - V_{n-1} over all R vectors as
 * one dense FP64 matrix product on the matrix cores, with the doubling-identity
 * dot products fused into the same kernel; the moments are formed as in
 * kpm_moments (mu_dev: device array of M doubles).  Real vectors only:
 * vec = KPM_VEC_RADEMACHER or KPM_VEC_UNIT (KPM_ERR_UNSUPPORTED otherwise).
 * H must be symmetric (not checked).  D <= 65536.  For D <= 128 the whole
 * recursion runs in one launch with H~ in on-chip memory, as long as its
 * per-step dot partials ((M/2 + 1) x ceil(R/16) x ceil(D/16) x 32 bytes) take
 * at most 256 MiB; otherwise one launch per step.  workspace_dev:
 * kpm_dense_workspace_bytes(D, M, R) bytes, 256-byte aligned (the padded H~,
 * the D x R vector blocks, partials and dots). */
size_t kpm_dense_workspace_bytes(int64_t D, int32_t M, int32_t R);
kpm_status kpm_dense_moments(const double *H_dev, int64_t D, double a, double b, int32_t M, int32_t R,
                             int32_t vec, uint64_t seed, uint64_t instance, void *workspace_dev,
                             size_t ws_bytes, double *mu_dev, void *stream);

/* Build the scaled operator H~ = (H - b)/a (Eq. (tilde)) in device memory that
 * the handle owns (one hipMalloc, released by kpm_free), in the recursion
 * precision `prec`.  The FP64 values are formed as d_i = (H_ii - b)/a and
 * H~_ij = (H_ij)/a; the FP32 operator rounds these.  a > 0 is required; the
 * caller is responsible for a and b enclosing the spectrum (see
 * kpm_scale_from_bounds).  Enqueues one kernel on `stream`.
 * Limits: N * (scalars per site) / 4 < 2^31; lattice extents < 2^31. */
kpm_status kpm_build(const kpm_ham_desc *desc, double a, double b, int32_t prec,
                     void *stream, kpm_ham **out);

/* Re-prepare an existing operator from new inputs of the same shape (same kind,
 * extents and hopping type; for CSR the same n, nnz and value type) and new
 * a, b, reusing its device memory: nothing is allocated, one kernel is
 * enqueued (CSR inputs are validated first, which synchronises the stream).
 * For Monte-Carlo loops over perturbed spin textures and for serving. */
kpm_status kpm_update(kpm_ham *h, const kpm_ham_desc *desc, double a, double b, void *stream);

/* Release the device memory kpm_build allocated for the operator H~ of
 * Eq. (tilde), and the handle itself.  The caller synchronises the streams
 * that used it first.  NULL is ignored. */
void kpm_free(kpm_ham *h);

/* The rescaling H~ = (H - b)/a (Eq. (tilde)) the operator was built or last
 * updated with: *a = alpha_-, *b = alpha_+ exactly as passed (no rounding of a
 * or b is applied in either precision).  KPM_ERR_INVALID_ARG for NULL. */
kpm_status kpm_ham_get_scale(const kpm_ham *h, double *a, double *b);

/* Number of sites N of the operator, or -1 for NULL. */
int64_t kpm_ham_dim(const kpm_ham *h);

/* alpha_-/alpha_+ of Eq. (tilde) from bounds, with a relative margin eps in [0, 1):
 *   a = (E_hi - E_lo)/(2 - eps),  b = (E_hi + E_lo)/2.   (Host arithmetic only.) */
kpm_status kpm_scale_from_bounds(double e_lo, double e_hi, double eps, double *a, double *b);

/* Bytes of device workspace one solve with M moments and R vectors needs:
 * the vector blocks of the recursion of Eq. (rn) (r_{n-1} and r_n, N x R
 * values each; four blocks for temporally blocked 2D solves), the per-work-item
 * partials of the dot products of Eq. (munr), and the floor(M/2) + 1 dot sums.
 * 0 on invalid arguments.  A pure host computation from the handle's shape. */
size_t kpm_workspace_bytes(const kpm_ham *h, int32_t M, int32_t R, int32_t vec);

/* All M moments mu_0..mu_{M-1} (Eq. (munr) through the doubling identities)
 * averaged over R start vectors of kind `vec`.  Runs floor(M/2) fused
 * recursion steps.  workspace_dev: device memory of at least
 * kpm_workspace_bytes(h, M, R, vec) bytes, 256-byte aligned, used as scratch
 * for the whole call (no other call may use it until the stream reaches the
 * end of this one).  mu_dev: device array of M doubles.  M >= 1, R >= 1. */
kpm_status kpm_moments(kpm_ham *h, int32_t M, int32_t R, int32_t vec, uint64_t seed,
                       uint64_t instance, void *workspace_dev, size_t ws_bytes,
                       double *mu_dev, void *stream);

/* kpm_moments without a caller workspace and without any allocation, for
 * callers that cannot allocate device memory (code under HIP graph capture,
 * serving loops or harnesses that forbid hipMalloc).  The workspace is the
 * library's own static device scratch of KPM_STATIC_SCRATCH_BYTES (64 MiB),
 * one copy per GPU, held from the library's load until the process ends; the
 * solve must fit it (kpm_workspace_bytes(h, M, R, vec) <= KPM_STATIC_SCRATCH_BYTES,
 * else KPM_ERR_WORKSPACE and nothing is enqueued).  The caller still passes the
 * operator and mu_dev[M].  No hipMalloc, hipFree or other allocating call is
 * made (the scratch address is looked up once per device, on that device's
 * first call).  Every call on one GPU shares its scratch and leaves its
 * contents behind (the solve writes each value before reading it, so nothing
 * needs clearing): calls that overlap on one GPU (other streams, other host
 * threads) race and must be serialised by the caller.  Results are bitwise
 * those of kpm_moments with the same arguments. */
#define KPM_STATIC_SCRATCH_BYTES (64u << 20)
size_t kpm_static_scratch_bytes(void);
kpm_status kpm_moments_static(kpm_ham *h, int32_t M, int32_t R, int32_t vec, uint64_t seed,
                              uint64_t instance, double *mu_dev, void *stream);

/* The same solve split into chunks, so that a caller can interleave other work
 * (serving) or stop and resume: begin draws r_0 and runs the first product;
 * advance runs up to max_steps further recursion steps and reports how many
 * remain; finish reduces the dot products and writes mu_dev[M].  The vector
 * state stays resident in the workspace between calls.  The handle is host
 * memory released by kpm_solve_free (which does not touch the workspace). */
kpm_status kpm_solve_begin(kpm_ham *h, int32_t M, int32_t R, int32_t vec, uint64_t seed,
                           uint64_t instance, void *workspace_dev, size_t ws_bytes,
                           void *stream, kpm_solve **out);
kpm_status kpm_solve_advance(kpm_solve *s, int32_t max_steps, void *stream, int32_t *remaining);
kpm_status kpm_solve_finish(kpm_solve *s, double *mu_dev, void *stream);
void kpm_solve_free(kpm_solve *s);
/* How the solve's recursion runs: 0 flat kernels (one step per launch), 1 march
 * kernels (one step per launch), 2 whole recursion in one workgroup (done at
 * begin), 3 temporal blocking (1 to 6 steps per launch, KPM_LAUNCH_TBLOCK);
 * -1 for NULL. */
int32_t kpm_solve_mode(const kpm_solve *s);

/* Many independent solves in one set of launches: each instance computes the
 * moments of Eq. (munr) by the recursion of Eq. (rn) exactly as kpm_moments
 * does (the paper runs one operator per launch; running many operators of
 * uneven size in shared launches is this library's extension).  Each
 * recursion step of every instance runs in one grid; the reduction partials
 * are per work item, so every instance's moments are bitwise equal to the same
 * solve run alone.  Instances run in waves whose state fits the Infinity Cache
 * (KPM_LAUNCH_WAVE_MIB).  Errors as kpm_moments; on an argument error nothing
 * is enqueued.  The workspace is kpm_workspace_bytes_batched bytes, 256-byte
 * aligned, caller-owned, and used until the stream reaches the end.  All
 * handles must share the recursion precision and, per launch group, the
 * operator class; mixed classes are grouped internally.  Arrays of length
 * `count`: h, M, R, seed, instance, mu_dev (device arrays of M[i] doubles). */
size_t kpm_workspace_bytes_batched(kpm_ham *const *h, int32_t count, const int32_t *M,
                                   const int32_t *R, int32_t vec);
kpm_status kpm_moments_batched(kpm_ham *const *h, int32_t count, const int32_t *M,
                               const int32_t *R, int32_t vec, const uint64_t *seed,
                               const uint64_t *instance, void *workspace_dev, size_t ws_bytes,
                               double *const *mu_dev, void *stream);

/* Steps a begun solve still has to run (0 once all floor(M/2) products are done). */
kpm_status kpm_solve_remaining(const kpm_solve *s, int32_t *remaining);

/* Host-only size query for admission control: device bytes that kpm_build plus one
 * solve of (M, R, vec) would occupy (operator + workspace); 0 on invalid input. */
size_t kpm_request_bytes(const kpm_ham_desc *desc, int32_t prec, int32_t M, int32_t R, int32_t vec);
/* Device bytes the operator of a built handle occupies. */
size_t kpm_ham_bytes(const kpm_ham *h);

/* Dynamic batches (continuous batching, for serving streams of requests): a set
 * of begun solves (kpm_solve_begin) that advance together.
 * kpm_batch_advance enqueues up to `steps` (<= 64) recursion steps in which
 * every launch covers all member solves of one operator class, each at its own
 * step n, so solves that joined at different times share launches; members
 * that have run all their steps are skipped.  Solves join (kpm_batch_add) and
 * leave (kpm_batch_remove) between calls; a solve that has left is finished
 * with kpm_solve_finish as usual.  Results are bitwise equal to the same solve
 * run alone (per-work-item partials).  All members share the recursion
 * precision.  The batch owns a small device table (one hipMalloc in create).
 * Calls on one batch must be serialised and use one stream.  kpm_batch_size
 * returns the number of members (-1 for NULL). */
typedef struct kpm_batch kpm_batch;
kpm_status kpm_batch_create(int32_t capacity, kpm_batch **out);
kpm_status kpm_batch_add(kpm_batch *b, kpm_solve *s);
kpm_status kpm_batch_remove(kpm_batch *b, kpm_solve *s);
int32_t kpm_batch_size(const kpm_batch *b);
kpm_status kpm_batch_advance(kpm_batch *b, int32_t steps, void *stream);
void kpm_batch_free(kpm_batch *b);

/* A whole batched solve (the same arguments as kpm_moments_batched) captured once
 * into a hipGraph on `stream` (a non-default stream) and replayed with one
 * kpm_graph_launch call: Monte-Carlo style loops re-prepare the operators with
 * kpm_update between replays and replay the same launch sequence (same seeds and
 * instances; the workspace and output arrays must stay valid for the graph's
 * life).  The capture contains kernels only (no memset or host copies). */
typedef struct kpm_graph kpm_graph;
kpm_status kpm_graph_capture_batched(kpm_ham *const *h, int32_t count, const int32_t *M, const int32_t *R,
                                     int32_t vec, const uint64_t *seed, const uint64_t *instance,
                                     void *workspace_dev, size_t ws_bytes, double *const *mu_dev,
                                     void *stream, kpm_graph **out);
kpm_status kpm_graph_launch(kpm_graph *g, void *stream);
void kpm_graph_free(kpm_graph *g);

/* Density of states, Eq. (fKPM), on the K first-kind Chebyshev points
 * x_k = cos(pi (k + 1/2)/K), k = 0..K-1, in FP64 on the device:
 *   rho(omega_k) = [g_0 mu_0 + 2 sum_{n=1}^{M-1} g_n mu_n cos(n theta_k)] / (pi a sin(theta_k)),
 *   omega_k = a x_k + b, with the Jackson coefficients
 *   g_n = [(M-n+1) cos(pi n/(M+1)) + sin(pi n/(M+1)) cot(pi/(M+1))]/(M+1)
 * when jackson != 0, else g_n = 1.  mu_dev[M], omega_dev[K], rho_dev[K]. */
kpm_status kpm_dos(const double *mu_dev, int32_t M, int32_t jackson, int32_t K, double a,
                   double b, double *omega_dev, double *rho_dev, void *stream);

/* Green's function from the moments of a start vector xi (per unit <xi|xi>):
 *   G(omega) = <xi|(omega + i0 - H)^{-1}|xi>,
 * expanded on the K first-kind Chebyshev points x_k = cos theta_k,
 * theta_k = pi (k + 1/2)/K, as
 *   G~(x) = -(i / sin theta) [g_0 mu_0 + 2 sum_{n>=1} g_n mu_n e^{-i n theta}],
 *   omega_k = a x_k + b,  G(omega_k) = G~(x_k)/a,
 * so Im G = -pi rho (Eq. (fKPM)) and Re G is its Hilbert transform.  The
 * kernel damps the truncation: KPM_KERNEL_NONE (g_n = 1), KPM_KERNEL_JACKSON,
 * KPM_KERNEL_LORENTZ (g_n = sinh(lambda (1 - n/M))/sinh(lambda), 0 < lambda <
 * 700; it broadens each level to a Lorentzian of half-width ~ lambda/M in
 * theta, the usual choice for Green's functions).  The paper names Green's
 * functions beside the DoS as targets of the expansion (Sec. I); with unit
 * start vectors at chosen sites (KPM_VEC_UNIT, R = 1, instance = site, one
 * batched solve per site) the moments are those of the local DoS and G is the
 * site-diagonal Green's function.  FP64; all arrays are device arrays
 * (omega, g_re, g_im of K doubles). */
typedef enum { KPM_KERNEL_NONE = 0, KPM_KERNEL_JACKSON = 1, KPM_KERNEL_LORENTZ = 2 } kpm_kernel;
kpm_status kpm_green(const double *mu_dev, int32_t M, int32_t kernel, double lambda, int32_t K,
                     double a, double b, double *omega_dev, double *g_re_dev, double *g_im_dev,
                     void *stream);

/* The start vectors r_0 exactly as the recursion draws them, in FP64, layout
 * [i][r] (real) or [i][r][2] (complex, re/im) with i < N, r < R.  complex_layout
 * selects the second layout (PHASE always produces complex values).  For tests. */
kpm_status kpm_start_vectors(int32_t vec, int32_t complex_layout, uint64_t seed,
                             uint64_t instance, int64_t N, int32_t R, double *out_dev,
                             void *stream);

/* Launch-shape tuning (host state, process-wide; applies to solves begun
 * afterwards).  Keys:
 *   KPM_LAUNCH_ELEMS_PER_THREAD  flat kernels: 16-byte chunks per thread per tile (1, 2 or 4)
 *   KPM_LAUNCH_MAX_BLOCKS        blocks per instance per launch (multiple of 8, >= 8; default
 *                                2048)
 *   KPM_LAUNCH_MARCH             1: lattices use the march kernels; 0: the flat kernels
 *   KPM_LAUNCH_MARCH_ITEMS       target work items per instance when the march axis is cut
 *                                into segments (fewer items -> longer segments; default 512).
 *                                FP32 3D spin solves whose vectors stream from HBM
 *                                (KPM_LAUNCH_STREAMING) take 4x this target on a quarter of
 *                                KPM_LAUNCH_MAX_BLOCKS blocks
 *   KPM_LAUNCH_XCD_SPLIT         how an instance's work items are split over the 8 XCDs:
 *                                0 automatic, 1 by column tiles, 2 by march segments, 3 none
 *   KPM_LAUNCH_ALTERNATE         1: odd march segments walk downwards
 *   KPM_LAUNCH_SMALL             1: a solve whose two vector blocks fit in the LDS of one
 *                                compute unit runs entirely in one workgroup (one launch)
 *   KPM_LAUNCH_STREAMING         march kernels: 1 = r_{n-1} read / r_{n+1} written with
 *                                non-temporal hints, 0 = cached, 2 (default) = cached when
 *                                vectors and operator take at most 256 MiB (they then
 *                                largely stay in the 256 MiB Infinity Cache between
 *                                steps), else 1
 *   KPM_LAUNCH_WAVE_MIB          kpm_moments_batched: instances run in waves, each wave
 *                                taking the next instances (in argument order) while their
 *                                vectors and operators total at most this many MiB (default
 *                                224, so a wave stays in the Infinity Cache); a wave runs all
 *                                its recursion steps before the next starts.  0 = one wave
 *   KPM_LAUNCH_TBLOCK            solves on 2D lattices (real or spin hopping; windows of
 *                                floor(512/Cg) sites of Cg <= 64 chunks each (KPM_LAUNCH_TB_GROUP),
 *                                L_x >= 512/Cg) take
 *                                several recursion steps per pass over the vectors (temporal
 *                                blocking; 4 vector buffers instead of 2, bitwise the same
 *                                vectors; in a dynamic batch they share blocked launches):
 *                                D = 3 .. 6: D steps per pass where at least D remain (only
 *                                r_{n+D-1} and r_{n+D} are written; x-tiles with D-site
 *                                halos, L_y >= 2D), shorter passes for the rest; -1
 *                                (default): D = 4 for FP32 real hopping and for FP32
 *                                spin hopping split into chunk groups, else 3; 1: two
 *                                steps per pass (L_y >= 4); 0: one step per pass.  D is
 *                                capped at 128/C (a quarter of the 512/C-site window);
 *                                below 2 the solve takes one step per pass.  Batched
 *                                solves (kpm_moments_batched) always take one step per
 *                                pass
 *   KPM_LAUNCH_TB3               solves on 3D lattices (KPM_LAUNCH_TBLOCK not 0) take two
 *                                recursion steps per pass (chunk-major vectors, row tiles
 *                                of whole planes, 4 vector buffers, bitwise the same
 *                                vectors; solo and dynamic batches): 1 for every 3D
 *                                lattice, -1 (default) for FP32 recursions with real
 *                                hopping only, 0 never.  Needs L_x L_y <= 1024 sites or
 *                                L_x <= 170
 *   KPM_LAUNCH_TB_GROUP          2D temporally blocked solves with more than 16 chunks per
 *                                site split its C chunks into groups of at least this many
 *                                chunks (default 8 = 128 bytes, 0 = one group), as many groups
 *                                as keep the window of floor(512 / chunks per group) sites
 *                                within L_x: a wider window recomputes and re-reads a smaller
 *                                halo share
 * The partial sums of the dot products are formed per work item, so the
 * moments do not depend on the grid (MAX_BLOCKS) nor on the batch an instance
 * runs in; the other keys change the work items and with them the order in
 * which rounding errors of the dot products are summed (well below 1e-15
 * relative).  Unknown keys or values return KPM_ERR_INVALID_ARG. */
typedef enum {
    KPM_LAUNCH_ELEMS_PER_THREAD = 0,
    KPM_LAUNCH_MAX_BLOCKS = 1,
    KPM_LAUNCH_MARCH = 2,
    KPM_LAUNCH_MARCH_ITEMS = 3,
    KPM_LAUNCH_XCD_SPLIT = 4,
    KPM_LAUNCH_ALTERNATE = 5,
    KPM_LAUNCH_SMALL = 6,
    KPM_LAUNCH_STREAMING = 7,
    KPM_LAUNCH_WAVE_MIB = 8,
    KPM_LAUNCH_TBLOCK = 9,
    KPM_LAUNCH_TB3 = 10,
    KPM_LAUNCH_TB_GROUP = 11
} kpm_launch_key;
kpm_status kpm_set_launch(int32_t key, int32_t value);
kpm_status kpm_get_launch(int32_t key, int32_t *value);

#ifdef __cplusplus
}
#endif

#endif /* KPM_H */
