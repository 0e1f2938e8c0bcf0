// libkpm: C ABI (include/kpm.h) over the gfx950 kernels in kpm_kernels.hpp.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "kpm.h"
#include "kpm_kernels.hpp"
#include "kpm_lanczos.hpp"
#include "kpm_dense.hpp"
#include "kpm_tblock.hpp"
#include "kpm_tblock3.hpp"

using namespace kpm;

namespace {

constexpr int PSLOTS_MAX = 64;          // ring slots of per-tile partials between reductions
int g_tpt = 4;                          // flat kernels: chunks per thread per tile
int g_max_blocks = 2048;                // blocks per instance per launch (multiple of 8)
int g_march = 1;                        // lattices use the march kernels
int g_march_items = 512;                // target work items per instance when choosing march segments
int g_xcd_split = 0;                    // 0 automatic, 1 by column tiles, 2 by segments, 3 none
int g_alternate = 1;                    // march: odd segments walk downwards
int g_small = 1;                        // solves whose two vector blocks fit in LDS run in one workgroup
int g_streaming = 2;                    // march: 0 cached, 1 non-temporal access of r_{n-1}/r_{n+1}, 2 by size
int g_wave_mib = 224;                   // batched solves: vectors + operators per wave (MiB), 0 = one wave
int g_tb3 = -1;                         // 3D lattices: two steps per pass: 0 off, 1 on, -1 FP32 real hopping only
int g_tblock = -1;                      // 2D lattices: steps per pass (temporal blocking): 0 one, 1 two, 3..6,
                                        // -1 by precision and hopping (tb_depth)
// Up to this much state (vectors + operator) r_{n+1} is stored cached, to be read back as r_n
// from the 256 MiB Infinity Cache; measured on 64 x 64 x L_z spin lattices (c64, R = 32),
// cached stores still win at 251 MiB (5.46 vs 5.00 TB/s; 234 MiB: 6.22 vs 5.01).
constexpr uint64_t CACHE_RESIDENT_BYTES = 256ull << 20;

// Dynamic LDS one workgroup may use for the small-solve path (0 if no device).
size_t small_lds_limit()
{
    static int cached_dev = -1;
    static size_t cached = 0;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (dev != cached_dev) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) v = 0;
        cached = v > 4096 ? (size_t)v - 4096 : 0;   // room for the static reduction scratch
        cached_dev = dev;
    }
    return cached;
}

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }
inline hipStream_t S(void *s) { return (hipStream_t)s; }

thread_local hipError_t g_last_hip = hipSuccess;   // last HIP error seen by this thread's calls

kpm_status check_launch()
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) g_last_hip = e;
    return e == hipSuccess ? KPM_OK : KPM_ERR_DEVICE;
}

// Phase factors w_j = e^{2 pi i 2^j / 2^30} (j = 0..29): angles 2 pi / 2^m for
// m = 1 (exactly -1), 2 (exactly i), then cos(t/2) = sqrt((1 + cos t)/2) and
// sin(t/2) = sin t / (2 cos(t/2)); w_j has m = 30 - j.  Uploaded to constant
// memory once per device before the first kernel that draws start vectors.
kpm_status ensure_phase_table()
{
    static std::mutex mu;
    static bool done[64] = {false};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return KPM_ERR_DEVICE;
    std::lock_guard<std::mutex> lock(mu);
    if (done[dev]) return KPM_OK;
    double w[PHASE_BITS][2];
    double c = -1.0, sn = 0.0;
    w[PHASE_BITS - 1][0] = c;
    w[PHASE_BITS - 1][1] = sn;
    c = 0.0;
    sn = 1.0;
    w[PHASE_BITS - 2][0] = c;
    w[PHASE_BITS - 2][1] = sn;
    for (int m = 3; m <= PHASE_BITS; ++m) {
        const double ch = std::sqrt((1.0 + c) / 2.0);
        const double sh = sn / (2.0 * ch);
        c = ch;
        sn = sh;
        w[PHASE_BITS - m][0] = c;
        w[PHASE_BITS - m][1] = sn;
    }
    if (hipMemcpyToSymbol(HIP_SYMBOL(kpm_phase_w), w, sizeof(w), 0, hipMemcpyHostToDevice) != hipSuccess)
        return KPM_ERR_DEVICE;
    done[dev] = true;
    return KPM_OK;
}

// ---------------------------------------------------------------------------
// small utility kernels
// ---------------------------------------------------------------------------
constexpr int UPLOAD_WORDS = 896;
struct UploadChunk {
    uint32_t n;
    uint32_t w[UPLOAD_WORDS];
};
__global__ void k_upload(uint32_t *dst, UploadChunk ch)
{
    for (uint32_t i = threadIdx.x; i < ch.n; i += blockDim.x) dst[i] = ch.w[i];
}

// Copy host bytes (multiple of 4) to device memory through kernel arguments,
// so the host buffer may be released as soon as this returns.
kpm_status upload(void *dst, const void *src, size_t bytes, hipStream_t st)
{
    const uint32_t *s = (const uint32_t *)src;
    uint32_t *d = (uint32_t *)dst;
    size_t words = bytes / 4;
    UploadChunk ch;
    for (size_t o = 0; o < words; o += UPLOAD_WORDS) {
        ch.n = (uint32_t)std::min((size_t)UPLOAD_WORDS, words - o);
        std::memcpy(ch.w, s + o, ch.n * 4);
        hipLaunchKernelGGL(k_upload, dim3(1), dim3(256), 0, st, d + o, ch);
    }
    return check_launch();
}

// ---------------------------------------------------------------------------
// operator preparation: H~ = (H - b)/a in the recursion precision
// ---------------------------------------------------------------------------
template <typename S>
__global__ __launch_bounds__(256) void k_prep_lattice(uint32_t Lx, uint32_t Ly, uint32_t Lz, int dim, int spin,
                                                      double t, double a, double b, const double *onsite,
                                                      const double *spinor, int has_diag, S *diag, S *bond, S *hop)
{
    const uint32_t N = Lx * Ly * Lz;
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) hop[0] = (S)((-t) / a);
    if (i >= N) return;
    if (has_diag) {
        const double eps = onsite ? onsite[i] : 0.0;
        diag[i] = (S)((eps - b) / a);
    }
    if (spin) {
        const uint32_t x = i % Lx, y = (i / Lx) % Ly, z = i / (Lx * Ly);
        const double ci = spinor[3 * (size_t)i], xi = spinor[3 * (size_t)i + 1], yi = spinor[3 * (size_t)i + 2];
        for (int ax = 0; ax < dim; ++ax) {
            uint32_t c[3] = {x, y, z};
            const uint32_t L[3] = {Lx, Ly, Lz};
            c[ax] = (c[ax] + 1) % L[ax];
            const uint32_t j = c[0] + Lx * (c[1] + Ly * c[2]);
            const double cj = spinor[3 * (size_t)j], xj = spinor[3 * (size_t)j + 1], yj = spinor[3 * (size_t)j + 2];
            // z = u_i^dag u_j
            const double zr = ci * cj + (xi * xj + yi * yj);
            const double zi = xi * yj - yi * xj;
            bond[((size_t)i * dim + ax) * 2] = (S)(((-t) * zr) / a);
            bond[((size_t)i * dim + ax) * 2 + 1] = (S)(((-t) * zi) / a);
        }
    }
}

// CSR structure checks: row_ptr must start at 0, end at nnz and not decrease;
// every column index must lie in [0, n).  Violations set *flag.
__global__ void k_zero_int(int *flag)
{
    if (threadIdx.x == 0) *flag = 0;
}
__global__ __launch_bounds__(256) void k_check_rowptr(int64_t n, int64_t nnz, const int64_t *row_ptr, int *flag)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i > n) return;
    const int64_t r = row_ptr[i];
    bool bad = (i == 0 && r != 0) || (i == n && r != nnz) || (i < n && r > row_ptr[i + 1]);
    if (bad) atomicOr(flag, 1);
}
__global__ __launch_bounds__(256) void k_check_cols(int64_t nnz, int64_t n, const int32_t *col, int *flag)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < nnz && (col[k] < 0 || (int64_t)col[k] >= n)) atomicOr(flag, 2);
}

template <typename S>
__global__ __launch_bounds__(256) void k_prep_csr(int64_t n, const int64_t *row_ptr, const int32_t *col,
                                                  const double *vre, const double *vim, double a, double b,
                                                  S *diag, S *val, int cplx)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double hii = 0.0;
    for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
        if (col[k] == i) {
            hii = hii + vre[k];
            if (cplx) {
                val[2 * k] = (S)0;
                val[2 * k + 1] = (S)0;
            } else {
                val[k] = (S)0;
            }
        } else if (cplx) {
            val[2 * k] = (S)(vre[k] / a);
            val[2 * k + 1] = (S)((vim ? vim[k] : 0.0) / a);
        } else {
            val[k] = (S)(vre[k] / a);
        }
    }
    diag[i] = (S)((hii - b) / a);
}

// ---------------------------------------------------------------------------
// Gershgorin bounds: exact min/max through order-preserving integer keys
// ---------------------------------------------------------------------------
__device__ __forceinline__ unsigned long long dkey(double x)
{
    unsigned long long u = (unsigned long long)__double_as_longlong(x);
    return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}
__device__ __forceinline__ double dunkey(unsigned long long k)
{
    unsigned long long u = (k >> 63) ? (k & 0x7fffffffffffffffull) : ~k;
    return __longlong_as_double((long long)u);
}
__global__ void k_bounds_init(unsigned long long *keys)
{
    if (threadIdx.x == 0) {
        keys[0] = dkey(INFINITY);
        keys[1] = dkey(-INFINITY);
    }
}
__global__ void k_bounds_decode(unsigned long long *keys)
{
    if (threadIdx.x == 0) {
        double lo = dunkey(keys[0]), hi = dunkey(keys[1]);
        ((double *)keys)[0] = lo;
        ((double *)keys)[1] = hi;
    }
}
__device__ __forceinline__ void bounds_commit(double lo, double hi, unsigned long long *keys)
{
    for (int off = 32; off > 0; off >>= 1) {
        lo = fmin(lo, __shfl_xor(lo, off, 64));
        hi = fmax(hi, __shfl_xor(hi, off, 64));
    }
    if ((threadIdx.x & 63) == 0) {
        atomicMin(&keys[0], dkey(lo));
        atomicMax(&keys[1], dkey(hi));
    }
}
__global__ __launch_bounds__(256) void k_bounds_lattice(uint32_t Lx, uint32_t Ly, uint32_t Lz, int dim, int spin,
                                                        double t, const double *onsite, const double *spinor,
                                                        unsigned long long *keys)
{
    const uint32_t N = Lx * Ly * Lz;
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    double lo = INFINITY, hi = -INFINITY;
    if (i < N) {
        const uint32_t x = i % Lx, y = (i / Lx) % Ly, z = i / (Lx * Ly);
        const uint32_t L[3] = {Lx, Ly, Lz};
        double rad = 0.0;
        for (int s = 0; s < 2 * dim; ++s) {
            if (!spin) {
                rad = rad + fabs(t);
            } else {
                uint32_t c[3] = {x, y, z};
                const int ax = s / 2;
                c[ax] = (s & 1) ? (c[ax] + 1) % L[ax] : (c[ax] + L[ax] - 1) % L[ax];
                const uint32_t j = c[0] + Lx * (c[1] + Ly * c[2]);
                const double ci = spinor[3 * (size_t)i], xi = spinor[3 * (size_t)i + 1], yi = spinor[3 * (size_t)i + 2];
                const double cj = spinor[3 * (size_t)j], xj = spinor[3 * (size_t)j + 1], yj = spinor[3 * (size_t)j + 2];
                const double zr = ci * cj + (xi * xj + yi * yj);
                const double zi = xi * yj - yi * xj;
                rad = rad + hypot((-t) * zr, (-t) * zi);
            }
        }
        const double eps = onsite ? onsite[i] : 0.0;
        lo = eps - rad;
        hi = eps + rad;
    }
    bounds_commit(lo, hi, keys);
}
__global__ __launch_bounds__(256) void k_bounds_csr(int64_t n, const int64_t *row_ptr, const int32_t *col,
                                                    const double *vre, const double *vim, unsigned long long *keys)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double lo = INFINITY, hi = -INFINITY;
    if (i < n) {
        double hii = 0.0, rad = 0.0;
        for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
            if (col[k] == i) hii = hii + vre[k];
            else rad = rad + hypot(vre[k], vim ? vim[k] : 0.0);
        }
        lo = hii - rad;
        hi = hii + rad;
    }
    bounds_commit(lo, hi, keys);
}

// ---------------------------------------------------------------------------
// density of states, Eq. (fKPM), one thread per Chebyshev point
// ---------------------------------------------------------------------------
constexpr int DOS_CHUNK = 2048;
// Kernel coefficient g_n of an M-moment expansion: 0 none, 1 Jackson
// [(M-n+1) cos(pi n/(M+1)) + sin(pi n/(M+1)) cot(pi/(M+1))]/(M+1),
// 2 Lorentz sinh(lam (1 - n/M))/sinh(lam).
__device__ inline double kernel_coef(int kind, int n, int M, double lam, double cot1)
{
    if (kind == 1) {
        const double x = (double)n / (double)(M + 1);
        return ((double)(M - n + 1) * cospi(x) + sinpi(x) * cot1) / (double)(M + 1);
    }
    if (kind == 2) return sinh(lam * (1.0 - (double)n / (double)M)) / sinh(lam);
    return 1.0;
}

// Sums over n of w_n cos(n theta_k) (and w_n sin(n theta_k) when `sine`),
// w_n = (2 - delta_n0) g_n mu_n, at the Chebyshev points theta_k = pi (k + 1/2)/K.
// A block of 256 threads takes DOS_PTS points: thread t works on point
// k = k0 + t % DOS_PTS and on the terms n = t / DOS_PTS (mod DOS_RES); the
// DOS_RES partial sums of a point are then added in a fixed order.  n theta_k
// is reduced exactly as pi m/(2K) with m = n (2k+1) mod 4K.  The w_n are
// staged through LDS in chunks.  Returns the sums for the calling thread's
// point in (fc, fs) on threads t < DOS_PTS (the others return zeros).
constexpr int DOS_PTS = 16;
constexpr int DOS_RES = 256 / DOS_PTS;
__device__ inline void chebyshev_sums(const double *mu, int M, int kind, double lam, int K, bool sine, double &fc,
                                      double &fs)
{
    __shared__ double w[DOS_CHUNK];
    __shared__ double red[2][DOS_RES][DOS_PTS];
    const int t = threadIdx.x, p = t % DOS_PTS, q = t / DOS_PTS;
    const int k = blockIdx.x * DOS_PTS + p;
    const uint64_t fourK = 4 * (uint64_t)K;
    const uint64_t step = (uint64_t)DOS_RES * (2 * (uint64_t)k + 1) % fourK;   // m advance per DOS_RES terms
    const double inv2K = 1.0 / (2.0 * (double)K);
    const double cot1 = cospi(1.0 / (double)(M + 1)) / sinpi(1.0 / (double)(M + 1));
    uint64_t m = (uint64_t)q * (2 * (uint64_t)k + 1) % fourK;                // m for n = q
    double c = 0.0, s = 0.0;
    for (int n0 = 0; n0 < M; n0 += DOS_CHUNK) {
        const int nn = min(DOS_CHUNK, M - n0);
        __syncthreads();
        for (int u = t; u < nn; u += blockDim.x) {
            const int n = n0 + u;
            w[u] = (n == 0 ? 1.0 : 2.0) * kernel_coef(kind, n, M, lam, cot1) * mu[n];
        }
        __syncthreads();
        if (k < K) {
            for (int u = q; u < nn; u += DOS_RES) {
                const double a = (double)m * inv2K;
                c += w[u] * cospi(a);
                if (sine) s += w[u] * sinpi(a);
                m += step;
                if (m >= fourK) m -= fourK;
            }
        }
    }
    red[0][q][p] = c;
    red[1][q][p] = s;
    __syncthreads();
    fc = 0.0;
    fs = 0.0;
    if (t < DOS_PTS)
        for (int r = 0; r < DOS_RES; ++r) {
            fc += red[0][r][t];
            fs += red[1][r][t];
        }
}

// density of states, Eq. (fKPM)
__global__ __launch_bounds__(256) void k_dos(const double *mu, int M, int jackson, int K, double a, double b,
                                             double *omega, double *rho)
{
    double f, unused;
    chebyshev_sums(mu, M, jackson ? 1 : 0, 0.0, K, false, f, unused);
    const int k = blockIdx.x * DOS_PTS + threadIdx.x;
    if (threadIdx.x < DOS_PTS && k < K) {
        const double th = ((double)k + 0.5) / (double)K;
        omega[k] = a * cospi(th) + b;
        rho[k] = f / (M_PI * sinpi(th)) / a;
    }
}

// Green's function G(omega + i0) = <xi|(omega + i0 - H)^{-1}|xi> from the
// moments: with x = cos theta, G~(x) = -(i/sin theta) sum_n w_n e^{-i n theta},
// G(omega) = G~(x)/a at omega = a x + b.
__global__ __launch_bounds__(256) void k_green(const double *mu, int M, int kind, double lam, int K, double a,
                                               double b, double *omega, double *gre, double *gim)
{
    double fc, fs;
    chebyshev_sums(mu, M, kind, lam, K, true, fc, fs);
    const int k = blockIdx.x * DOS_PTS + threadIdx.x;
    if (threadIdx.x < DOS_PTS && k < K) {
        const double th = ((double)k + 0.5) / (double)K;
        const double sn = sinpi(th);
        omega[k] = a * cospi(th) + b;
        gre[k] = -fs / sn / a;
        gim[k] = -fc / sn / a;
    }
}

// start vectors exported in FP64 for tests
__global__ __launch_bounds__(256) void k_export_start(int vec, int cplx, uint64_t seed, uint64_t instance, uint32_t N,
                                                      uint32_t R, double *out)
{
    const uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (uint64_t)N * R) return;
    const uint32_t i = (uint32_t)(e / R), r = (uint32_t)(e % R);
    uint64_t w[4] = {0, 0, 0, 0};
    if (vec != VEC_UNIT) start_words(seed, instance, i, r / 4, w);
    double re, im;
    start_value(vec, w[r & 3], instance, N, i, r, re, im);
    if (cplx) {
        out[2 * e] = re;
        out[2 * e + 1] = im;
    } else {
        out[e] = re;
    }
}

// ---------------------------------------------------------------------------
// kernel tables by (precision, operator kind, chunks per thread)
// ---------------------------------------------------------------------------
typedef void (*step_fn)(const Inst *, const uint32_t *, int32_t);
typedef void (*init_fn)(const Inst *, const uint32_t *);

// Kernel class of a solve: one launch covers instances of one class.
inline int kernel_key(int opk, int mode, int wide, int nt) { return ((opk * 4 + mode) * 2 + wide) * 2 + nt; }

template <typename S, bool WIDE, bool NT>
step_fn march_for(int opk)
{
    switch (opk) {
    case OP_REAL2: return k_step_march<S, OP_REAL2, WIDE, NT>;
    case OP_REAL3: return k_step_march<S, OP_REAL3, WIDE, NT>;
    case OP_SPIN2: return k_step_march<S, OP_SPIN2, WIDE, NT>;
    default: return k_step_march<S, OP_SPIN3, WIDE, NT>;
    }
}
template <typename S, bool WIDE>
step_fn step_for(int opk, int mode, int nt)
{
    if (mode == MODE_MARCH) return nt ? march_for<S, WIDE, true>(opk) : march_for<S, WIDE, false>(opk);
    switch (opk) {
    case OP_REAL2: return k_step_flat<S, OP_REAL2, WIDE>;
    case OP_REAL3: return k_step_flat<S, OP_REAL3, WIDE>;
    case OP_SPIN2: return k_step_flat<S, OP_SPIN2, WIDE>;
    case OP_SPIN3: return k_step_flat<S, OP_SPIN3, WIDE>;
    case OP_CSR_R: return k_step_flat<S, OP_CSR_R, WIDE>;
    default: return k_step_flat<S, OP_CSR_C, WIDE>;
    }
}
step_fn get_step(int prec, int opk, int mode, int wide, int nt)
{
    if (prec == KPM_F64) return wide ? step_for<double, true>(opk, mode, nt) : step_for<double, false>(opk, mode, nt);
    return wide ? step_for<float, true>(opk, mode, nt) : step_for<float, false>(opk, mode, nt);
}
init_fn get_init(int prec, int wide)
{
    if (prec == KPM_F64) return wide ? k_init<double, true> : k_init<double, false>;
    return wide ? k_init<float, true> : k_init<float, false>;
}

}  // namespace

// ---------------------------------------------------------------------------
// handles
// ---------------------------------------------------------------------------
struct kpm_ham {
    int32_t kind, hop, prec, dim, opk;
    int64_t L[3];
    int64_t N, nnz;
    double a, b, t;
    int cplx_op, has_diag;
    char *mem;
    size_t mem_bytes;
    void *diag, *bond, *hopv, *val;
    int64_t *row_ptr;
    int32_t *col;
    int *flag;
};

struct kpm_solve {
    kpm_ham *h;
    Inst inst;
    int wide;
    char *ws;
    Inst *tab_dev;
    int32_t next;      // next recursion step n to run
    int32_t written;   // dots indices [0, written) have partials
    int32_t reduced;   // dots indices [0, reduced) are reduced
    uint64_t state;    // bytes the recursion touches per step (vectors + operator)
    void *tbuf[4];     // temporal blocking: the four vector buffers
    int tb_prev, tb_cur;   // ... and which of them hold r_{next-1}, r_next
};

namespace {

// Geometry of one solve: everything but device pointers.
struct Plan {
    int cplx, mode, wide, xcd, alt, nt;
    uint32_t W, Rs, C, nel, tiles, nb;
    uint32_t P, Lm, S, nct, nseg;
    int32_t K, P_slots, tpt;
    size_t esz;
    size_t part_bytes, dots_bytes, buf_bytes;
    uint32_t nbuf;    // vector buffers (2, or 4 with temporal blocking)
    uint32_t tbg;     // 2D temporal blocking: chunk groups per site
    int32_t tbh;      // temporal blocking: x-tile halo = steps of the deepest pass (1 .. 6)
    uint64_t state;   // bytes the recursion touches per step (vectors + operator)
    uint32_t grid_cap;   // most blocks per launch (0: KPM_LAUNCH_MAX_BLOCKS)
};

// Halo (= steps of the deepest pass, 2 for pairs) of a temporally blocked solve.
// Default (-1), measured on 2048^2 lattices: FP32 real hopping four steps (R = 64: 2.5x
// one step per pass); FP32 spin hopping three (R = 16 / 32: 1.53x / 1.68x, 1-10% faster
// than four) unless its sites are split into chunk groups (grouped), where four are
// 2.4-5.6% faster (us per step, three -> four: 2048^2 R = 64 684.1 -> 653.9, 1024^2
// R = 48 163.4 -> 159.1, R = 64 195.7 -> 191.0, 512^2 R = 64 71.0 -> 67.0); FP64 three
// (four need over 150 VGPRs and run slower; spin R = 8: 1.27x).
int tb_depth(int prec, int opk, bool grouped = false)
{
    if (g_tblock < 0) return (prec == KPM_F64 || (opk == OP_SPIN2 && !grouped)) ? 3 : 4;
    return g_tblock >= 3 ? g_tblock : 2;
}
// The halo actually used with C chunks per site (in groups or not): at most a quarter
// of the window of TB_BLOCK / C sites, so that at least half of it is owned.
int tb_halo(int prec, int opk, uint32_t C, bool grouped = false)
{
    return std::min<int>(tb_depth(prec, opk, grouped), (int)(TB_BLOCK / C / 4));
}

// Chunk groups of a 2D blocked solve whose window would be narrower than 32
// sites (more than 16 chunks per site): the most groups (the widest window, so
// the smallest halo share) that keep at least g_tb_group chunks (128 bytes at
// 8) per site in a group and a window no wider than the row.  0 turns grouping
// off.  Measured on the 2048^2 lattice, R = 64: FP64 (32 chunks, window 16 ->
// 64 sites) 1443 -> 1306 ms per solve; FP32 (16 chunks, window 32 -> 64) 478 ->
// 506 ms, hence no grouping from 32-site windows up.
int g_tb_group = 8;
uint32_t tb_groups(uint32_t C, uint32_t Lx)
{
    uint32_t best = 1;
    if (g_tb_group <= 0 || TB_BLOCK / C >= 32) return best;
    for (uint32_t G = 2; G <= C; ++G) {
        if (C % G) continue;
        const uint32_t Cg = C / G;
        if (Cg < (uint32_t)g_tb_group || Lx < TB_BLOCK / Cg) break;
        best = G;
    }
    return best;
}

// Store kind for r_{n+1}: it is read again as r_n by the next step, so keep it
// cached when everything the recursion touches per step (all instances of a
// batch together) fits the Infinity Cache, and stream it past the caches
// otherwise.
int stream_choice(uint64_t state_bytes)
{
    return g_streaming == 2 ? (state_bytes > CACHE_RESIDENT_BYTES ? 1 : 0) : g_streaming;
}

// Tiling of a 3D lattice for two-step passes (chunk-major vectors): row tiles
// of T owned rows plus two rows of r_n each side (or the whole plane), at most
// TB3_TILE elements; segments of at least 4 planes, as many as keep the work
// items within one block per compute unit (TB3_ITEMS).  False when a row tile
// cannot hold two owned rows.
constexpr uint32_t TB3_ITEMS = 512;
bool tb3_plan(const kpm_ham *h, Plan &p)
{
    const uint32_t Lx = (uint32_t)h->L[0], Ly = (uint32_t)h->L[1], Lz = (uint32_t)h->L[2];
    uint32_t nty = 1, Ty = Ly;
    if ((uint64_t)Lx * Ly > TB3_TILE) {
        if (TB3_TILE / Lx < 6) return false;
        const uint32_t rmax = TB3_TILE / Lx - 4;
        nty = (Ly + rmax - 1) / rmax;
        Ty = (Ly + nty - 1) / nty;
    }
    const uint64_t units = (uint64_t)p.C * nty;
    uint32_t nseg = (uint32_t)std::max<uint64_t>(1, TB3_ITEMS / units);
    nseg = std::max<uint32_t>(1, std::min<uint32_t>(nseg, std::max<uint32_t>(1, Lz / 4)));
    p.S = (Lz + nseg - 1) / nseg;
    p.nseg = (Lz + p.S - 1) / p.S;
    p.P = Ty;
    p.nct = nty;
    p.Lm = Lz;
    p.tiles = (uint32_t)(units * p.nseg);
    // all chunks of a segment on one XCD (they share its bonds and diagonal in L2)
    p.xcd = p.nseg >= 8 ? 2 : 0;
    return true;
}

bool make_plan(const kpm_ham *h, int32_t M, int32_t R, int32_t vec, Plan &p, bool allow_tb = true)
{
    if (!h || M < 1 || R < 1 || vec < 0 || vec > 2) return false;
    std::memset(&p, 0, sizeof(p));
    p.esz = h->prec == KPM_F64 ? 8 : 4;
    p.W = (uint32_t)(16 / p.esz);
    p.cplx = (h->cplx_op || vec == KPM_VEC_PHASE) ? 1 : 0;
    const uint64_t scal = (uint64_t)R * (p.cplx ? 2 : 1);
    const uint64_t Rs = (scal + p.W - 1) / p.W * p.W;
    const uint64_t C = Rs / p.W;
    const uint64_t nel = (uint64_t)h->N * C;
    if (Rs > (1u << 30) || nel >= (1ull << 31) - (1ull << 16)) return false;
    p.Rs = (uint32_t)Rs;
    p.C = (uint32_t)C;
    p.nel = (uint32_t)nel;
    p.tpt = g_tpt;
    // byte offsets beyond 32 bits need the 64-bit addressing variant
    const uint64_t bond_bytes = (uint64_t)h->N * (h->dim ? h->dim : 1) * 2 * p.esz;
    p.wide = (nel * 16 >= (1ull << 32) || bond_bytes >= (1ull << 32)) ? 1 : 0;
    const uint64_t small_bytes = 2ull * nel * 16;
    p.nbuf = 2;
    if (g_small && small_bytes <= small_lds_limit()) {
        p.mode = MODE_SMALL;
        p.tiles = SMALL_WAVES;   // per-wave dot partials
        p.xcd = 0;
    } else if (allow_tb && g_tblock && g_march && (h->opk == OP_REAL2 || h->opk == OP_SPIN2) &&
               tb_halo(h->prec, h->opk, p.C / tb_groups(p.C, (uint32_t)h->L[0]),
                       tb_groups(p.C, (uint32_t)h->L[0]) > 1) >= 2 &&
               h->L[0] >= TB_BLOCK / (p.C / tb_groups(p.C, (uint32_t)h->L[0])) &&
               h->L[1] >= 2 * tb_halo(h->prec, h->opk, p.C / tb_groups(p.C, (uint32_t)h->L[0]),
                                      tb_groups(p.C, (uint32_t)h->L[0]) > 1)) {
        // several steps per pass: the site's chunks in tbg groups, windows of
        // floor(TB_BLOCK/Cg) sites of one group (Cg = C/tbg; threads beyond window * Cg
        // idle), x-tiles of the window less 2 tbh halo sites, segments of rows
        p.mode = MODE_TB;
        p.nbuf = 4;
        p.tbg = tb_groups(p.C, (uint32_t)h->L[0]);
        const uint32_t Cg = p.C / p.tbg;
        p.tbh = tb_halo(h->prec, h->opk, Cg, p.tbg > 1);
        const uint32_t Tn = TB_BLOCK / Cg - 2 * (uint32_t)p.tbh;
        p.P = (uint32_t)h->L[0];
        p.Lm = (uint32_t)h->L[1];
        p.nct = (p.P + Tn - 1) / Tn;
        // more and shorter segments than the one-step kernels (6x the item target;
        // measured on the 2048^2 lattice with two-step passes: 4096 items 455 us per
        // step, 512 items 554 us; with four-step passes (R = 64) 1024 / 1536 / 2048 /
        // 2560 / 3072 / 4096 items: 524.7 / 491.9 / 471.5 / 469.5 / 466.8 / 476.4 ms
        // per solve, FP64 three-step passes 1428.7 / 1349.4 / 1303.5 / 1277.6 / 1281.7
        // / 1302.4 ms)
        const uint64_t units = (uint64_t)p.nct * p.tbg;
        const uint64_t target = 6ull * (uint64_t)g_march_items;
        uint32_t nseg = (uint32_t)((target + units - 1) / units);
        nseg = std::max<uint32_t>(1, std::min<uint32_t>(nseg, std::max<uint32_t>(1, p.Lm / 8)));
        p.S = (p.Lm + nseg - 1) / nseg;
        p.nseg = (p.Lm + p.S - 1) / p.S;
        p.tiles = (uint32_t)(units * p.nseg);
        p.xcd = units >= 8 ? 1 : 0;
    } else if (allow_tb && g_tblock && g_march &&
               (g_tb3 > 0 ? (h->opk == OP_REAL3 || h->opk == OP_SPIN3)
                          : (g_tb3 < 0 && h->opk == OP_REAL3 && h->prec == KPM_F32)) &&
               tb3_plan(h, p)) {
        p.mode = MODE_TB3;
        p.nbuf = 4;
        p.tbh = 2;
    } else if (h->dim && g_march) {
        p.mode = MODE_MARCH;
        p.P = (uint32_t)(h->dim == 3 ? h->L[0] * h->L[1] : h->L[0]);
        p.Lm = (uint32_t)(h->dim == 3 ? h->L[2] : h->L[1]);
        const uint64_t PC = (uint64_t)p.P * p.C;
        p.nct = (uint32_t)((PC + BLOCK - 1) / BLOCK);
        // FP32 3D spin hopping whose vectors stream from HBM: 4x the item target
        // (shorter segments) on a quarter of the blocks
        const bool spin_stream = h->opk == OP_SPIN3 && h->prec == KPM_F32 &&
                                 stream_choice(2ull * h->N * p.Rs * p.esz + (uint64_t)h->N * 7 * p.esz) == 1;
        p.grid_cap = spin_stream ? std::max<uint32_t>(8, (uint32_t)g_max_blocks / 32 * 8) : (uint32_t)g_max_blocks;
        const uint64_t items = spin_stream ? 4ull * (uint64_t)g_march_items : (uint64_t)g_march_items;
        uint32_t nseg = (uint32_t)((items + p.nct - 1) / p.nct);
        nseg = std::max<uint32_t>(1, std::min<uint32_t>(nseg, std::max<uint32_t>(1, p.Lm / 8)));
        p.S = (p.Lm + nseg - 1) / nseg;
        p.nseg = (p.Lm + p.S - 1) / p.S;
        p.tiles = p.nct * p.nseg;
        // split per XCD along the column tiles (measured best on the 64^3 and
        // 2048^2 lattices), else along the march segments
        p.xcd = p.nct >= XCD_MIN_ITEMS ? 1 : ((p.nseg >= 8 && p.tiles >= XCD_MIN_ITEMS) ? 2 : 0);
        if (g_xcd_split == 1) p.xcd = p.nct >= XCD_MIN_ITEMS ? 1 : 0;
        if (g_xcd_split == 2) p.xcd = p.nseg >= 8 ? 2 : 0;
        if (g_xcd_split == 3) p.xcd = 0;
        p.alt = g_alternate;
    } else {
        p.mode = MODE_FLAT;
        const uint64_t per_tile = (uint64_t)BLOCK * p.tpt;
        p.tiles = (uint32_t)((nel + per_tile - 1) / per_tile);
        p.xcd = p.tiles >= XCD_MIN_ITEMS ? 1 : 0;
    }
    const uint32_t nb = (p.tiles + 7) / 8 * 8;
    p.nb = std::min<uint32_t>(nb, p.grid_cap ? p.grid_cap : (uint32_t)g_max_blocks);
    p.K = M / 2;
    p.P_slots = std::min(p.K + 1, PSLOTS_MAX);
    p.part_bytes = align256((size_t)p.P_slots * p.tiles * 4 * sizeof(double));
    p.dots_bytes = align256((size_t)(p.K + 1) * 4 * sizeof(double));
    p.buf_bytes = align256((size_t)h->N * p.Rs * p.esz);
    if (p.mode == MODE_SMALL) {
        // one launch runs every step: a partial slot per step, reduced afterwards
        p.P_slots = p.K + 1;
        p.part_bytes = align256((size_t)p.P_slots * p.tiles * 4 * sizeof(double));
        p.buf_bytes = 0;
        p.nb = 1;
    }
    // r_{n+1} is read again as r_n by the next step: keep it cached when the
    // whole state fits the Infinity Cache, stream it otherwise
    p.state = 2ull * p.buf_bytes + (uint64_t)h->N * (h->dim ? (1 + 2 * h->dim) : 1) * p.esz;
    p.nt = stream_choice(p.state);
    return true;
}

size_t instance_bytes(const Plan &p) { return p.part_bytes + p.dots_bytes + p.nbuf * p.buf_bytes; }

void fill_inst(const kpm_ham *h, const Plan &p, int32_t M, int32_t R, int32_t vec, uint64_t seed, uint64_t instance,
               char *region, Inst &I)
{
    std::memset(&I, 0, sizeof(I));
    I.opk = h->opk;
    I.has_diag = h->has_diag;
    I.Lx = (uint32_t)h->L[0];
    I.Ly = (uint32_t)h->L[1];
    I.Lz = (uint32_t)h->L[2];
    I.N = (uint32_t)h->N;
    I.fLx = make_fastdiv(I.Lx ? I.Lx : 1);
    I.fLy = make_fastdiv(I.Ly ? I.Ly : 1);
    I.fC = make_fastdiv(p.C);
    I.C = p.C;
    I.Rs = p.Rs;
    I.nel = p.nel;
    I.tiles = p.tiles;
    I.nb = p.nb;
    I.block0 = 0;
    I.bstride = 1;
    I.tpt = p.tpt;
    I.mode = p.mode;
    I.xcd = p.xcd;
    I.alt = p.alt;
    I.nt = p.nt;
    I.P = p.P;
    I.Lm = p.Lm;
    I.S = p.S;
    I.nct = p.nct;
    I.nseg = p.nseg;
    I.cplx = p.cplx;
    I.M = M;
    I.K = p.K;
    I.R = R;
    I.vec = vec;
    I.step0 = 0;
    I.pslots = p.P_slots;
    I.tbh = p.tbh;
    I.tbg = p.tbg ? p.tbg : 1;
    I.seed = seed;
    I.instance = instance;
    I.norm = (vec == KPM_VEC_UNIT) ? (double)R : (double)h->N * (double)R;
    I.diag = h->diag;
    I.bond = h->bond;
    I.hop = h->hopv;
    I.row_ptr = h->row_ptr;
    I.col = h->col;
    I.val = h->val;
    I.partial = (double *)region;
    I.dots = (double *)(region + p.part_bytes);
    I.buf0 = region + p.part_bytes + p.dots_bytes;
    I.buf1 = region + p.part_bytes + p.dots_bytes + p.buf_bytes;
    I.mu = nullptr;
}

kpm_status launch_init_tb(int prec, int wide, const Inst *tab, uint32_t blocks, void *cur, hipStream_t st)
{
    typedef void (*fn)(const Inst *, void *);
    static const fn fns[2][2] = {{k_init_tb<double, false>, k_init_tb<double, true>},
                                 {k_init_tb<float, false>, k_init_tb<float, true>}};
    hipLaunchKernelGGL(fns[prec == KPM_F64 ? 0 : 1][wide ? 1 : 0], dim3(blocks), dim3(TB_BLOCK), 0, st, tab, cur);
    return check_launch();
}

kpm_status launch_init_tb3(int prec, int wide, const Inst *tab, uint32_t blocks, void *cur, hipStream_t st)
{
    typedef void (*fn)(const Inst *, void *);
    static const fn fns[2][2] = {{k_init_tb3<double, false>, k_init_tb3<double, true>},
                                 {k_init_tb3<float, false>, k_init_tb3<float, true>}};
    hipLaunchKernelGGL(fns[prec == KPM_F64 ? 0 : 1][wide ? 1 : 0], dim3(blocks), dim3(TB3_BLOCK), 0, st, tab, cur);
    return check_launch();
}

// one- and two-step passes of the 3D blocked kernel (solo: tab[0] at step arg with
// the given buffers; batched: pass arg of the block map's instances, -1 = remainder)
typedef void (*tb3_fn)(const Inst *, const uint32_t *, int32_t, const void *, const void *, void *, void *);
template <typename S, int OPK, int D>
tb3_fn tb3_pick(int wide, int nt)
{
    return wide ? (nt ? k_step_tb3<S, OPK, true, true, D> : k_step_tb3<S, OPK, true, false, D>)
                : (nt ? k_step_tb3<S, OPK, false, true, D> : k_step_tb3<S, OPK, false, false, D>);
}
template <int D>
tb3_fn tb3_for(int prec, int opk, int wide, int nt)
{
    if (opk == OP_SPIN3)
        return prec == KPM_F64 ? tb3_pick<double, OP_SPIN3, D>(wide, nt) : tb3_pick<float, OP_SPIN3, D>(wide, nt);
    return prec == KPM_F64 ? tb3_pick<double, OP_REAL3, D>(wide, nt) : tb3_pick<float, OP_REAL3, D>(wide, nt);
}
kpm_status launch_tb3(int depth, int prec, int opk, int wide, int nt, const Inst *tab, const uint32_t *bmap,
                      uint32_t blocks, int32_t arg, const void *prev, const void *cur, void *outa, void *outb,
                      hipStream_t st)
{
    if ((opk != OP_REAL3 && opk != OP_SPIN3) || depth < 1 || depth > 2) return KPM_ERR_INVALID_ARG;
    tb3_fn f = depth == 2 ? tb3_for<2>(prec, opk, wide, nt) : tb3_for<1>(prec, opk, wide, nt);
    hipLaunchKernelGGL(f, dim3(blocks), dim3(TB3_BLOCK), 0, st, tab, bmap, arg, prev, cur, outa, outb);
    return check_launch();
}
// A pass of a blocked solve of either kind.
kpm_status launch_pass(int mode, int depth, int prec, int opk, int wide, int nt, const Inst *tab, const uint32_t *bmap,
                       uint32_t blocks, int32_t arg, const void *prev, const void *cur, void *outa, void *outb,
                       hipStream_t st);

// depth-D passes (D = 1 .. 6) of the temporally blocked kernel, real or spin hopping
typedef void (*tbd_fn)(const Inst *, const uint32_t *, int32_t, const void *, const void *, void *, void *);
template <typename S, int OPK, int D>
tbd_fn tbd_pick(int wide, int nt)
{
    return wide ? (nt ? k_step_tbd<S, OPK, true, true, D> : k_step_tbd<S, OPK, true, false, D>)
                : (nt ? k_step_tbd<S, OPK, false, true, D> : k_step_tbd<S, OPK, false, false, D>);
}
template <int D>
tbd_fn tbd_for(int prec, int opk, int wide, int nt)
{
    if (opk == OP_SPIN2)
        return prec == KPM_F64 ? tbd_pick<double, OP_SPIN2, D>(wide, nt) : tbd_pick<float, OP_SPIN2, D>(wide, nt);
    return prec == KPM_F64 ? tbd_pick<double, OP_REAL2, D>(wide, nt) : tbd_pick<float, OP_REAL2, D>(wide, nt);
}
// Solo: tab[0] at step arg with the given buffers (bmap = nullptr).  Batched: the
// instances of the block map run pass arg of their chunk (arg = -1: their
// remainder pass of this depth), buffers from the table.
kpm_status launch_tbd(int depth, int prec, int opk, int wide, int nt, const Inst *tab, const uint32_t *bmap,
                      uint32_t blocks, int32_t arg, const void *prev, const void *cur, void *outa, void *outb,
                      hipStream_t st)
{
    if (opk != OP_REAL2 && opk != OP_SPIN2) return KPM_ERR_INVALID_ARG;
    tbd_fn f = nullptr;
    switch (depth) {
    case 1: f = tbd_for<1>(prec, opk, wide, nt); break;
    case 2: f = tbd_for<2>(prec, opk, wide, nt); break;
    case 3: f = tbd_for<3>(prec, opk, wide, nt); break;
    case 4: f = tbd_for<4>(prec, opk, wide, nt); break;
    case 5: f = tbd_for<5>(prec, opk, wide, nt); break;
    case 6: f = tbd_for<6>(prec, opk, wide, nt); break;
    default: return KPM_ERR_INVALID_ARG;
    }
    hipLaunchKernelGGL(f, dim3(blocks), dim3(TB_BLOCK), 0, st, tab, bmap, arg, prev, cur, outa, outb);
    return check_launch();
}

kpm_status launch_pass(int mode, int depth, int prec, int opk, int wide, int nt, const Inst *tab, const uint32_t *bmap,
                       uint32_t blocks, int32_t arg, const void *prev, const void *cur, void *outa, void *outb,
                       hipStream_t st)
{
    if (mode == MODE_TB3) return launch_tb3(depth, prec, opk, wide, nt, tab, bmap, blocks, arg, prev, cur, outa, outb, st);
    return launch_tbd(depth, prec, opk, wide, nt, tab, bmap, blocks, arg, prev, cur, outa, outb, st);
}

kpm_status launch_init(int prec, int wide, const Inst *tab, const uint32_t *bmap, uint32_t blocks, hipStream_t st)
{
    hipLaunchKernelGGL(get_init(prec, wide), dim3(blocks), dim3(BLOCK), 0, st, tab, bmap);
    return check_launch();
}
kpm_status launch_step(int prec, int opk, int mode, int wide, int nt, const Inst *tab, const uint32_t *bmap,
                       uint32_t blocks, int32_t k, hipStream_t st)
{
    hipLaunchKernelGGL(get_step(prec, opk, mode, wide, nt), dim3(blocks), dim3(BLOCK), 0, st, tab, bmap, k);
    return check_launch();
}
typedef void (*small_fn)(const Inst *);
template <typename S>
small_fn small_for(int opk)
{
    switch (opk) {
    case OP_REAL2: return k_solve_small<S, OP_REAL2>;
    case OP_REAL3: return k_solve_small<S, OP_REAL3>;
    case OP_SPIN2: return k_solve_small<S, OP_SPIN2>;
    case OP_SPIN3: return k_solve_small<S, OP_SPIN3>;
    case OP_CSR_R: return k_solve_small<S, OP_CSR_R>;
    default: return k_solve_small<S, OP_CSR_C>;
    }
}
// `count` small solves of one operator class, one workgroup each, with
// `lds` bytes of dynamic LDS (the largest of the group).
kpm_status launch_small(int prec, int opk, const Inst *tab, uint32_t count, size_t lds, hipStream_t st)
{
    small_fn f = prec == KPM_F64 ? small_for<double>(opk) : small_for<float>(opk);
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) != hipSuccess) return KPM_ERR_DEVICE;
    if (cs == hipStreamCaptureStatusNone &&
        hipFuncSetAttribute((const void *)f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)small_lds_limit()) !=
            hipSuccess)
        return KPM_ERR_DEVICE;
    hipLaunchKernelGGL(f, dim3(count), dim3(SMALL_BLOCK), lds, st, tab);
    return check_launch();
}

kpm_status launch_reduce(const Inst *tab, int32_t count, int32_t klo, int32_t nk, hipStream_t st)
{
    if (nk <= 0) return KPM_OK;
    hipLaunchKernelGGL(k_reduce, dim3(nk, count), dim3(BLOCK), 0, st, tab, klo, nk);
    return check_launch();
}
kpm_status launch_moments(const Inst *tab, int32_t count, int32_t Mmax, hipStream_t st)
{
    hipLaunchKernelGGL(k_moments, dim3((Mmax + BLOCK - 1) / BLOCK, count), dim3(BLOCK), 0, st, tab);
    return check_launch();
}

// Validate CSR structure on the device (synchronises `st`); flag_dev: one device int.
kpm_status validate_csr(const kpm_ham_desc *d, int *flag_dev, hipStream_t st)
{
    hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(64), 0, st, flag_dev);
    hipLaunchKernelGGL(k_check_rowptr, dim3((uint32_t)((d->n + 1 + 255) / 256)), dim3(256), 0, st, d->n, d->nnz,
                       d->row_ptr_dev, flag_dev);
    int flag = 0;
    if (hipMemcpyAsync(&flag, flag_dev, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess) return KPM_ERR_DEVICE;
    if (hipStreamSynchronize(st) != hipSuccess) return KPM_ERR_DEVICE;
    if (flag) return KPM_ERR_INVALID_ARG;
    if (d->nnz > 0) {
        hipLaunchKernelGGL(k_check_cols, dim3((uint32_t)((d->nnz + 255) / 256)), dim3(256), 0, st, d->nnz, d->n,
                           d->col_dev, flag_dev);
        if (hipMemcpyAsync(&flag, flag_dev, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess) return KPM_ERR_DEVICE;
        if (hipStreamSynchronize(st) != hipSuccess) return KPM_ERR_DEVICE;
        if (flag) return KPM_ERR_INVALID_ARG;
    }
    return check_launch();
}

bool valid_desc(const kpm_ham_desc *d)
{
    if (!d) return false;
    if (d->kind == KPM_SQUARE_2D || d->kind == KPM_CUBIC_3D) {
        const int dim = d->kind == KPM_CUBIC_3D ? 3 : 2;
        for (int k = 0; k < dim; ++k)
            if (d->L[k] < 1 || d->L[k] >= (1ll << 31)) return false;
        const int64_t Lz = dim == 3 ? d->L[2] : 1;
        const double N = (double)d->L[0] * (double)d->L[1] * (double)Lz;
        if (N >= 2147483648.0) return false;
        if (d->hop != KPM_HOP_REAL && d->hop != KPM_HOP_SPIN) return false;
        if (d->hop == KPM_HOP_SPIN && !d->spinor_dev) return false;
        return std::isfinite(d->t);
    }
    if (d->kind == KPM_CSR) {
        return d->n >= 1 && d->n < (1ll << 31) && d->nnz >= 0 && d->row_ptr_dev && (d->nnz == 0 || (d->col_dev && d->val_re_dev));
    }
    return false;
}

}  // namespace

extern "C" {

const char *kpm_last_hip_error(void) { return hipGetErrorString(g_last_hip); }

const char *kpm_status_string(kpm_status st)
{
    switch (st) {
    case KPM_OK: return "ok";
    case KPM_ERR_INVALID_ARG: return "invalid argument";
    case KPM_ERR_OUT_OF_MEMORY: return "out of device memory";
    case KPM_ERR_DEVICE: return "HIP runtime error";
    case KPM_ERR_BOUNDS: return "spectrum outside [-1, 1] or divergence";
    case KPM_ERR_UNSUPPORTED: return "size not supported";
    case KPM_ERR_WORKSPACE: return "workspace missing or too small";
    }
    return "unknown status";
}

kpm_status kpm_scale_from_bounds(double e_lo, double e_hi, double eps, double *a, double *b)
{
    if (!a || !b || !(e_hi > e_lo) || !(eps >= 0.0 && eps < 1.0) || !std::isfinite(e_lo) || !std::isfinite(e_hi))
        return KPM_ERR_INVALID_ARG;
    *a = (e_hi - e_lo) / (2.0 - eps);
    *b = (e_hi + e_lo) / 2.0;
    return KPM_OK;
}

kpm_status kpm_bounds_gershgorin(const kpm_ham_desc *d, double *bounds_dev, void *stream)
{
    if (!valid_desc(d) || !bounds_dev) return KPM_ERR_INVALID_ARG;
    hipStream_t st = S(stream);
    unsigned long long *keys = (unsigned long long *)bounds_dev;
    if (d->kind == KPM_CSR) {
        kpm_status v = validate_csr(d, (int *)bounds_dev, st);
        if (v != KPM_OK) return v;
        hipLaunchKernelGGL(k_bounds_init, dim3(1), dim3(64), 0, st, keys);
        const uint32_t blocks = (uint32_t)((d->n + 255) / 256);
        hipLaunchKernelGGL(k_bounds_csr, dim3(blocks), dim3(256), 0, st, d->n, d->row_ptr_dev, d->col_dev,
                           d->val_re_dev, d->val_im_dev, keys);
    } else {
        const int dim = d->kind == KPM_CUBIC_3D ? 3 : 2;
        const uint32_t Lz = dim == 3 ? (uint32_t)d->L[2] : 1u;
        const uint64_t N = (uint64_t)d->L[0] * d->L[1] * Lz;
        hipLaunchKernelGGL(k_bounds_init, dim3(1), dim3(64), 0, st, keys);
        hipLaunchKernelGGL(k_bounds_lattice, dim3((uint32_t)((N + 255) / 256)), dim3(256), 0, st, (uint32_t)d->L[0],
                           (uint32_t)d->L[1], Lz, dim, d->hop == KPM_HOP_SPIN ? 1 : 0, d->t, d->onsite_dev,
                           d->spinor_dev, keys);
    }
    hipLaunchKernelGGL(k_bounds_decode, dim3(1), dim3(64), 0, st, keys);
    return check_launch();
}

// Launch the preparation kernel(s) of H~ = (H - b)/a into the handle's memory.
static kpm_status prep_launch(kpm_ham *h, const kpm_ham_desc *d, double a, double b, hipStream_t st)
{
    h->a = a;
    h->b = b;
    h->t = d->t;
    const uint32_t blocks = (uint32_t)((h->N + 255) / 256);
    if (h->kind == KPM_CSR) {
        kpm_status v = validate_csr(d, h->flag, st);
        if (v != KPM_OK) return v;
        hipError_t ce = hipMemcpyAsync(h->row_ptr, d->row_ptr_dev, (size_t)(h->N + 1) * 8, hipMemcpyDeviceToDevice, st);
        if (ce == hipSuccess && h->nnz)
            ce = hipMemcpyAsync(h->col, d->col_dev, (size_t)h->nnz * 4, hipMemcpyDeviceToDevice, st);
        if (ce != hipSuccess) return KPM_ERR_DEVICE;
        if (h->prec == KPM_F64)
            hipLaunchKernelGGL(k_prep_csr<double>, dim3(blocks), dim3(256), 0, st, h->N, d->row_ptr_dev, d->col_dev,
                               d->val_re_dev, d->val_im_dev, a, b, (double *)h->diag, (double *)h->val, h->cplx_op);
        else
            hipLaunchKernelGGL(k_prep_csr<float>, dim3(blocks), dim3(256), 0, st, h->N, d->row_ptr_dev, d->col_dev,
                               d->val_re_dev, d->val_im_dev, a, b, (float *)h->diag, (float *)h->val, h->cplx_op);
    } else {
        const int spin = d->hop == KPM_HOP_SPIN;
        // d_i = (H_ii - b)/a vanishes identically when there is no on-site term and b == 0
        h->has_diag = (d->onsite_dev != nullptr || b != 0.0) ? 1 : 0;
        if (h->prec == KPM_F64)
            hipLaunchKernelGGL(k_prep_lattice<double>, dim3(blocks), dim3(256), 0, st, (uint32_t)h->L[0],
                               (uint32_t)h->L[1], (uint32_t)h->L[2], h->dim, spin, d->t, a, b, d->onsite_dev,
                               d->spinor_dev, h->has_diag, (double *)h->diag, (double *)h->bond, (double *)h->hopv);
        else
            hipLaunchKernelGGL(k_prep_lattice<float>, dim3(blocks), dim3(256), 0, st, (uint32_t)h->L[0],
                               (uint32_t)h->L[1], (uint32_t)h->L[2], h->dim, spin, d->t, a, b, d->onsite_dev,
                               d->spinor_dev, h->has_diag, (float *)h->diag, (float *)h->bond, (float *)h->hopv);
    }
    return check_launch();
}

// Geometry and device-memory layout of the operator (no allocation).
struct HamLayout {
    size_t o_diag, o_val, o_rp, o_col, o_flag, o_hop, o_bond, bytes;
};
static void ham_layout(const kpm_ham_desc *d, int32_t prec, kpm_ham &h, HamLayout &L)
{
    std::memset(&L, 0, sizeof(L));
    h.kind = d->kind;
    h.hop = d->hop;
    h.prec = prec;
    const size_t esz = prec == KPM_F64 ? 8 : 4;
    if (d->kind == KPM_CSR) {
        h.dim = 0;
        h.N = d->n;
        h.nnz = d->nnz;
        h.L[0] = d->n; h.L[1] = 1; h.L[2] = 1;
        h.cplx_op = d->val_im_dev ? 1 : 0;
        h.opk = h.cplx_op ? OP_CSR_C : OP_CSR_R;
        h.has_diag = 1;
        L.o_diag = 0;
        L.o_val = align256(L.o_diag + h.N * esz);
        L.o_rp = align256(L.o_val + (size_t)h.nnz * esz * (h.cplx_op ? 2 : 1));
        L.o_col = align256(L.o_rp + (size_t)(h.N + 1) * 8);
        L.o_flag = align256(L.o_col + (size_t)h.nnz * 4 + 4);
        L.bytes = L.o_flag + 256;
    } else {
        h.dim = d->kind == KPM_CUBIC_3D ? 3 : 2;
        h.L[0] = d->L[0];
        h.L[1] = d->L[1];
        h.L[2] = h.dim == 3 ? d->L[2] : 1;
        h.N = h.L[0] * h.L[1] * h.L[2];
        const int spin = d->hop == KPM_HOP_SPIN;
        h.cplx_op = spin;
        h.opk = spin ? (h.dim == 3 ? OP_SPIN3 : OP_SPIN2) : (h.dim == 3 ? OP_REAL3 : OP_REAL2);
        L.o_hop = 0;
        L.o_diag = 256;
        L.o_bond = align256(L.o_diag + h.N * esz);
        L.bytes = align256(L.o_bond + (spin ? (size_t)h.N * h.dim * 2 * esz : 0)) + 256;
    }
}

kpm_status kpm_build(const kpm_ham_desc *d, double a, double b, int32_t prec, void *stream, kpm_ham **out)
{
    if (!out || !valid_desc(d) || !(a > 0.0) || !std::isfinite(a) || !std::isfinite(b) ||
        (prec != KPM_F64 && prec != KPM_F32))
        return KPM_ERR_INVALID_ARG;
    hipStream_t st = S(stream);
    kpm_ham *h = new (std::nothrow) kpm_ham();
    if (!h) return KPM_ERR_OUT_OF_MEMORY;
    HamLayout L;
    ham_layout(d, prec, *h, L);
    if (hipError_t me = hipMalloc((void **)&h->mem, L.bytes); me != hipSuccess) {
        g_last_hip = me;
        delete h;
        return KPM_ERR_OUT_OF_MEMORY;
    }
    h->mem_bytes = L.bytes;
    if (d->kind == KPM_CSR) {
        h->diag = h->mem + L.o_diag;
        h->val = h->mem + L.o_val;
        h->row_ptr = (int64_t *)(h->mem + L.o_rp);
        h->col = (int32_t *)(h->mem + L.o_col);
        h->flag = (int *)(h->mem + L.o_flag);
    } else {
        h->hopv = h->mem + L.o_hop;
        h->diag = h->mem + L.o_diag;
        h->bond = h->cplx_op ? h->mem + L.o_bond : nullptr;
    }
    kpm_status s = prep_launch(h, d, a, b, st);
    if (s != KPM_OK) {
        (void)hipFree(h->mem);
        delete h;
        return s;
    }
    *out = h;
    return KPM_OK;
}

size_t kpm_request_bytes(const kpm_ham_desc *d, int32_t prec, int32_t M, int32_t R, int32_t vec)
{
    if (!valid_desc(d) || (prec != KPM_F64 && prec != KPM_F32)) return 0;
    kpm_ham h;
    std::memset(&h, 0, sizeof(h));
    HamLayout L;
    ham_layout(d, prec, h, L);
    Plan p;
    if (!make_plan(&h, M, R, vec, p)) return 0;
    return L.bytes + align256(sizeof(Inst)) + instance_bytes(p);
}

size_t kpm_ham_bytes(const kpm_ham *h) { return h ? h->mem_bytes : 0; }

kpm_status kpm_update(kpm_ham *h, const kpm_ham_desc *d, double a, double b, void *stream)
{
    if (!h || !valid_desc(d) || !(a > 0.0) || !std::isfinite(a) || !std::isfinite(b) || d->kind != h->kind)
        return KPM_ERR_INVALID_ARG;
    if (d->kind == KPM_CSR) {
        if (d->n != h->N || d->nnz != h->nnz || (d->val_im_dev ? 1 : 0) != h->cplx_op) return KPM_ERR_INVALID_ARG;
    } else {
        const int dim = d->kind == KPM_CUBIC_3D ? 3 : 2;
        if (d->L[0] != h->L[0] || d->L[1] != h->L[1] || (dim == 3 && d->L[2] != h->L[2]) || d->hop != h->hop)
            return KPM_ERR_INVALID_ARG;
    }
    return prep_launch(h, d, a, b, S(stream));
}

void kpm_free(kpm_ham *h)
{
    if (!h) return;
    if (h->mem) (void)hipFree(h->mem);
    delete h;
}

int64_t kpm_ham_dim(const kpm_ham *h) { return h ? h->N : -1; }

kpm_status kpm_ham_get_scale(const kpm_ham *h, double *a, double *b)
{
    if (!h || !a || !b) return KPM_ERR_INVALID_ARG;
    *a = h->a;
    *b = h->b;
    return KPM_OK;
}

size_t kpm_workspace_bytes(const kpm_ham *h, int32_t M, int32_t R, int32_t vec)
{
    Plan p;
    if (!make_plan(h, M, R, vec, p)) return 0;
    return align256(sizeof(Inst)) + instance_bytes(p);
}

kpm_status kpm_solve_begin(kpm_ham *h, int32_t M, int32_t R, int32_t vec, uint64_t seed, uint64_t instance,
                           void *ws, size_t ws_bytes, void *stream, kpm_solve **out)
{
    Plan p;
    if (!out || !make_plan(h, M, R, vec, p)) return KPM_ERR_INVALID_ARG;
    const size_t need = align256(sizeof(Inst)) + instance_bytes(p);
    if (!ws || ((uintptr_t)ws & 255) || ws_bytes < need) return KPM_ERR_WORKSPACE;
    if (ensure_phase_table() != KPM_OK) return KPM_ERR_DEVICE;
    kpm_solve *s = new (std::nothrow) kpm_solve();
    if (!s) return KPM_ERR_OUT_OF_MEMORY;
    hipStream_t st = S(stream);
    s->h = h;
    s->state = p.state;
    s->ws = (char *)ws;
    s->tab_dev = (Inst *)ws;
    fill_inst(h, p, M, R, vec, seed, instance, s->ws + align256(sizeof(Inst)), s->inst);
    kpm_status e = upload(s->tab_dev, &s->inst, sizeof(Inst), st);
    s->wide = p.wide;
    if (p.mode == MODE_SMALL) {
        // the whole recursion runs now; its partials are reduced by finish
        if (e == KPM_OK) e = launch_small(h->prec, h->opk, s->tab_dev, 1, 2 * (size_t)p.nel * 16, st);
        s->next = p.K;
        s->written = p.K + 1;
        s->reduced = 0;
        if (e != KPM_OK) {
            delete s;
            return e;
        }
        *out = s;
        return KPM_OK;
    }
    if (p.mode == MODE_TB || p.mode == MODE_TB3) {
        // four vector buffers; r_0 goes to buffer 1 (buffer 0 plays r_{-1}, never read)
        char *b = s->ws + align256(sizeof(Inst)) + p.part_bytes + p.dots_bytes;
        for (int q = 0; q < 4; ++q) s->tbuf[q] = b + (size_t)q * p.buf_bytes;
        s->inst.buf0 = s->tbuf[0];
        s->inst.buf1 = s->tbuf[1];
        s->inst.tb2 = s->tbuf[2];
        s->inst.tb3 = s->tbuf[3];
        s->tb_prev = 0;
        s->tb_cur = 1;
        if (e == KPM_OK)
            e = p.mode == MODE_TB3 ? launch_init_tb3(h->prec, p.wide, s->tab_dev, p.nb, s->tbuf[1], st)
                                   : launch_init_tb(h->prec, p.wide, s->tab_dev, p.nb, s->tbuf[1], st);
        s->written = 1;
        s->reduced = 0;
        s->next = 0;
        if (e != KPM_OK) {
            delete s;
            return e;
        }
        *out = s;
        return KPM_OK;
    }
    if (e == KPM_OK) e = launch_init(h->prec, p.wide, s->tab_dev, nullptr, p.nb, st);
    s->written = 1;
    s->reduced = 0;
    s->next = 0;
    if (e == KPM_OK && p.K >= 1) {
        e = launch_step(h->prec, h->opk, p.mode, p.wide, p.nt, s->tab_dev, nullptr, p.nb, 0, st);
        s->next = 1;
        s->written = 2;
    }
    if (e != KPM_OK) {
        delete s;
        return e;
    }
    *out = s;
    return KPM_OK;
}

// Temporal blocking: the two buffers of four not holding (r_{n-1}, r_n), ascending.
static void tb_free(int prev, int cur, int f[2])
{
    int nf = 0;
    for (int q = 0; q < 4; ++q)
        if (q != prev && q != cur) f[nf++] = q;
}
// Buffer roles after a pass of `depth` steps: depth >= 2 leaves (r_{n+depth-1},
// r_{n+depth}) in the free buffers (ascending); one step leaves r_{n+1} in the
// lower free buffer.  The batched kernel derives the same roles in-kernel.
static void tb_rotate(int &prev, int &cur, int depth)
{
    int f[2];
    tb_free(prev, cur, f);
    if (depth >= 2) {
        prev = f[0];
        cur = f[1];
    } else {
        prev = cur;
        cur = f[0];
    }
}

static kpm_status solve_reduce_pending(kpm_solve *s, hipStream_t st)
{
    const int32_t n = s->written - s->reduced;
    if (n <= 0) return KPM_OK;
    // dots index idx = step0 + 1 + k with step0 = 0
    kpm_status e = launch_reduce(s->tab_dev, 1, s->reduced - 1, n, st);
    s->reduced = s->written;
    return e;
}

kpm_status kpm_solve_advance(kpm_solve *s, int32_t max_steps, void *stream, int32_t *remaining)
{
    if (!s || max_steps < 0) return KPM_ERR_INVALID_ARG;
    hipStream_t st = S(stream);
    const Inst &I = s->inst;
    kpm_status e = KPM_OK;
    if (I.mode == MODE_TB || I.mode == MODE_TB3) {
        // passes of tbh steps (the tiles' halo); a shorter one for the remainder or a
        // smaller budget
        int32_t done = 0;
        while (done < max_steps && s->next < I.K && e == KPM_OK) {
            const int32_t adv = std::min(std::min(I.K - s->next, max_steps - done), I.tbh);
            if (s->written - s->reduced + adv > I.pslots) e = solve_reduce_pending(s, st);
            if (e != KPM_OK) break;
            int f[2];
            tb_free(s->tb_prev, s->tb_cur, f);
            // r_{n+adv-1}, r_{n+adv} into the free buffers, which become (prev, cur); a single
            // step writes r_{n+1} alone
            e = launch_pass(I.mode, adv, s->h->prec, s->h->opk, s->wide, I.nt, s->tab_dev, nullptr, I.nb, s->next,
                            s->tbuf[s->tb_prev], s->tbuf[s->tb_cur], s->tbuf[adv >= 2 ? f[0] : f[1]],
                            s->tbuf[adv >= 2 ? f[1] : f[0]], st);
            tb_rotate(s->tb_prev, s->tb_cur, adv);
            s->next += adv;
            s->written += adv;
            done += adv;
        }
        if (e == KPM_OK && s->written - s->reduced >= I.pslots) e = solve_reduce_pending(s, st);
        if (remaining) *remaining = I.K - s->next;
        return e;
    }
    for (int32_t c = 0; c < max_steps && s->next < I.K && e == KPM_OK; ++c) {
        if (s->written - s->reduced >= I.pslots) e = solve_reduce_pending(s, st);
        if (e != KPM_OK) break;
        e = launch_step(s->h->prec, I.opk, I.mode, s->wide, I.nt, s->tab_dev, nullptr, I.nb, s->next, st);
        s->next += 1;
        s->written += 1;
    }
    if (e == KPM_OK && s->written - s->reduced >= I.pslots) e = solve_reduce_pending(s, st);
    if (remaining) *remaining = I.K - s->next;
    return e;
}

kpm_status kpm_solve_finish(kpm_solve *s, double *mu_dev, void *stream)
{
    if (!s || !mu_dev) return KPM_ERR_INVALID_ARG;
    hipStream_t st = S(stream);
    kpm_status e = KPM_OK;
    if (s->next < s->inst.K) e = kpm_solve_advance(s, s->inst.K - s->next, stream, nullptr);
    if (e == KPM_OK) e = solve_reduce_pending(s, st);
    if (e != KPM_OK) return e;
    s->inst.mu = mu_dev;
    e = upload(s->tab_dev, &s->inst, sizeof(Inst), st);
    if (e == KPM_OK) e = launch_moments(s->tab_dev, 1, s->inst.M, st);
    return e;
}

void kpm_solve_free(kpm_solve *s) { delete s; }

int32_t kpm_solve_mode(const kpm_solve *s) { return s ? s->inst.mode : -1; }

kpm_status kpm_moments(kpm_ham *h, int32_t M, int32_t R, int32_t vec, uint64_t seed, uint64_t instance, void *ws,
                       size_t ws_bytes, double *mu_dev, void *stream)
{
    if (!mu_dev) return KPM_ERR_INVALID_ARG;
    kpm_solve *s = nullptr;
    kpm_status e = kpm_solve_begin(h, M, R, vec, seed, instance, ws, ws_bytes, stream, &s);
    if (e != KPM_OK) return e;
    e = kpm_solve_finish(s, mu_dev, stream);
    kpm_solve_free(s);
    return e;
}

// ---------------------------------------------------------------------------
// the same solve with the library's own device scratch (no allocation)
// ---------------------------------------------------------------------------
namespace {
// One copy per device, held from the code object's load until the process ends.
__device__ __align__(256) char scratch[KPM_STATIC_SCRATCH_BYTES];

// Device address of this device's copy of `scratch`, looked up once per device with
// that device current.  In host code the name `scratch` is only a host-side stand-in:
// kernels and copies must be given this address instead.
kpm_status scratch_address(void **out)
{
    static std::mutex mu;
    static void *addr[64] = {nullptr};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return KPM_ERR_DEVICE;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            g_last_hip = e != hipSuccess ? e : hipErrorInvalidSymbol;
            return KPM_ERR_DEVICE;
        }
        addr[dev] = p;
    }
    *out = addr[dev];
    return KPM_OK;
}
}  // namespace

size_t kpm_static_scratch_bytes(void) { return (size_t)KPM_STATIC_SCRATCH_BYTES; }

kpm_status kpm_moments_static(kpm_ham *h, int32_t M, int32_t R, int32_t vec, uint64_t seed, uint64_t instance,
                              double *mu_dev, void *stream)
{
    if (!h || !mu_dev) return KPM_ERR_INVALID_ARG;
    const size_t need = kpm_workspace_bytes(h, M, R, vec);
    if (need == 0) return KPM_ERR_INVALID_ARG;
    if (need > (size_t)KPM_STATIC_SCRATCH_BYTES) return KPM_ERR_WORKSPACE;
    void *ws = nullptr;
    const kpm_status e = scratch_address(&ws);
    if (e != KPM_OK) return e;
    // the solve writes every value of its workspace before reading it, so the
    // previous call's contents need no clearing
    return kpm_moments(h, M, R, vec, seed, instance, ws, (size_t)KPM_STATIC_SCRATCH_BYTES, mu_dev, stream);
}

// ---------------------------------------------------------------------------
// batched solves
// ---------------------------------------------------------------------------
namespace {
// Block placement of one launch group (instances of one kernel class, in table
// order).  Instances whose work is split per XCD take contiguous, 8-aligned
// block ranges (every nb is a multiple of 8).  When there are at least 8 of
// the others they are balanced over the XCDs: largest first (by chunks, i.e.
// work), each goes whole to the least loaded XCD if that stays within 10% of
// an even share, and is otherwise split per XCD like the big ones (when it has
// at least SPLIT_MIN_UNITS units to split).  The instances of XCD x take its blocks x, x + 8,
// x + 16, ... one after another (block stride 8), so all blocks of such an
// instance run on one XCD and the halo planes its neighbouring column tiles
// fetch stay in that XCD's L2.  Fewer than 8 are placed contiguously, so each
// still spreads over the whole chip.  Splitting changes only which block runs
// a work item, never the items, so results do not depend on the placement.
// Writes block0/bstride (and xcd for split instances) into the instances and
// the per-block map (instance index within the group, NO_INSTANCE for idle
// blocks); returns the grid size.
//
// The waves of a static batch (wave = true) run many instances through all
// their steps together: there, with at least 8 instances, one-step march
// instances are balanced whole over the XCDs even where their own plan would
// split them (all column tiles of an instance then share one L2 for their
// in-plane neighbour reads), with 25% slack over the even share before one is
// split.  Measured on the batch of 256 spin cubes (L = 16 .. 48): 193.6 ->
// 183.7 ms per batched solve (only the instances without a split of their own,
// 10% slack: 192.3 ms).  Dynamic batches, whose few members differ widely in
// size, measured 1-2% slower under that rule and keep the one above.
constexpr uint32_t SPLIT_MIN_UNITS = 48;   // below this a split leaves too few units per XCD (halo re-fetch)
uint32_t place_blocks(std::vector<Inst> &ins, std::vector<uint32_t> &map, bool wave = false)
{
    std::vector<uint32_t> big, small;
    for (uint32_t r = 0; r < ins.size(); ++r)
        ((wave && ins.size() >= 8 && ins[r].mode == MODE_MARCH) || !ins[r].xcd ? small : big).push_back(r);
    if (small.size() < 8) {
        big.insert(big.end(), small.begin(), small.end());
        std::sort(big.begin(), big.end());
        small.clear();
    }
    for (uint32_t r : small) ins[r].xcd = 0;
    auto cost = [&](uint32_t r) { return ins[r].nel ? (uint64_t)ins[r].nel : (uint64_t)ins[r].nb; };
    auto units = [&](uint32_t r) {
        if (ins[r].mode == MODE_TB3) return ins[r].nct * ins[r].C;
        if (ins[r].mode == MODE_TB) return ins[r].nct * ins[r].tbg;
        return ins[r].mode == MODE_MARCH ? ins[r].nct : ins[r].tiles;
    };
    std::stable_sort(small.begin(), small.end(), [&](uint32_t a, uint32_t b) { return cost(a) > cost(b); });
    uint64_t total = 0;
    for (uint32_t r : small) total += cost(r);
    const double share = (double)total / 8.0 * (wave ? 1.25 : 1.10);
    uint64_t load[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    uint32_t used[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    std::vector<uint32_t> whole, xcd_of;
    for (uint32_t r : small) {
        int x = 0;
        for (int y = 1; y < 8; ++y)
            if (load[y] < load[x]) x = y;
        if ((double)(load[x] + cost(r)) > share && units(r) >= SPLIT_MIN_UNITS && ins[r].nb >= 8) {
            ins[r].xcd = 1;   // split over all XCDs by units
            big.push_back(r);
            for (int y = 0; y < 8; ++y) load[y] += cost(r) / 8;
            continue;
        }
        whole.push_back(r);
        xcd_of.push_back((uint32_t)x);
        load[x] += cost(r);
        used[x] += ins[r].nb;
    }
    uint32_t blocks = 0;
    for (uint32_t r : big) {
        ins[r].block0 = blocks;
        ins[r].bstride = 1;
        for (uint32_t j = 0; j < ins[r].nb; ++j) map.push_back(r);
        blocks += ins[r].nb;
    }
    if (whole.empty()) return blocks;
    uint32_t span = 0;
    for (int x = 0; x < 8; ++x) span = std::max(span, used[x]);
    const size_t base = map.size();
    map.resize(base + 8 * (size_t)span, NO_INSTANCE);
    uint32_t off[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (size_t q = 0; q < whole.size(); ++q) {
        const uint32_t r = whole[q], x = xcd_of[q];
        Inst &I = ins[r];
        I.block0 = blocks + x + 8 * off[x];
        I.bstride = 8;
        for (uint32_t j = 0; j < I.nb; ++j) map[base + x + 8 * (size_t)(off[x] + j)] = r;
        off[x] += I.nb;
    }
    return blocks + 8 * span;
}
}  // namespace
namespace {
// One multi-instance launch: the instances of one kernel class, contiguous in
// the table, with their block map.
struct BatchGroup {
    int opk, mode, wide, nt;
    uint32_t first, count;   // table range
    uint32_t blocks;         // grid size
    size_t map_off;          // offset into the block map (words)
    size_t lds;              // single-workgroup solves: dynamic LDS bytes
};
// Instances whose recursions run together, step by step, before the next wave
// starts.  A wave's vectors and operators are sized to stay in the Infinity
// Cache between steps.
struct BatchWave {
    uint32_t first, count;   // table range
    int32_t Kmax;
    std::vector<BatchGroup> groups;
};
struct BatchLayout {
    std::vector<Plan> plans;
    std::vector<int> order;           // table index -> instance
    std::vector<BatchGroup> small;    // single-workgroup solves, one launch per kernel class
    std::vector<BatchWave> waves;
    size_t tab_off, map_off, inst_off, total, map_words;
    std::vector<size_t> region_off;   // per instance
    int prec;
};

// Appends the groups of instances `ids` (one per kernel class, in order of
// first appearance) to `groups`, their instances to L.order, and sizes their
// block maps.
void add_groups(kpm_ham *const *h, const std::vector<int> &ids, BatchLayout &L, std::vector<BatchGroup> &groups)
{
    std::vector<int> keys;
    for (int i : ids) {
        const int key = kernel_key(h[i]->opk, L.plans[i].mode, L.plans[i].wide, L.plans[i].nt);
        if (std::find(keys.begin(), keys.end(), key) == keys.end()) keys.push_back(key);
    }
    for (int key : keys) {
        BatchGroup g{0, 0, 0, 0, (uint32_t)L.order.size(), 0, 0, L.map_words, 0};
        std::vector<Inst> ins;
        for (int i : ids) {
            const Plan &p = L.plans[i];
            if (kernel_key(h[i]->opk, p.mode, p.wide, p.nt) != key) continue;
            g.opk = h[i]->opk;
            g.mode = p.mode;
            g.wide = p.wide;
            g.nt = p.nt;
            g.lds = std::max(g.lds, 2 * (size_t)p.nel * 16);
            Inst I;
            std::memset(&I, 0, sizeof(I));
            I.nb = p.nb;
            I.xcd = p.xcd;
            I.nel = p.nel;
            I.mode = p.mode;
            I.nct = p.nct;
            I.tiles = p.tiles;
            ins.push_back(I);
            L.order.push_back(i);
        }
        g.count = (uint32_t)ins.size();
        if (g.mode != MODE_SMALL) {
            std::vector<uint32_t> m;
            g.blocks = place_blocks(ins, m, true);
            L.map_words += m.size();
        }
        groups.push_back(g);
    }
}

bool batch_layout(kpm_ham *const *h, int32_t count, const int32_t *M, const int32_t *R, int32_t vec, BatchLayout &L)
{
    if (!h || count < 1 || count > 65535 || !M || !R) return false;
    L.plans.resize(count);
    L.prec = h[0] ? h[0]->prec : -1;
    L.map_words = 0;
    std::vector<int> small, rest;
    for (int i = 0; i < count; ++i) {
        if (!h[i] || h[i]->prec != L.prec) return false;
        if (!make_plan(h[i], M[i], R[i], vec, L.plans[i], false)) return false;
        if (L.plans[i].mode == MODE_SMALL) {
            small.push_back(i);
        } else {
            rest.push_back(i);
        }
    }
    // Waves: consecutive instances (argument order) while their state stays
    // within wave_bytes.  (Dealing the instances out to the waves by size
    // measured slower on batches of equal cubes, 834 vs 677 us per step for
    // 2560 cubes of 16^3.)
    const uint64_t wave_bytes = (uint64_t)g_wave_mib << 20;
    std::vector<std::vector<int>> waves;
    {
        uint64_t ws = 0;
        for (int i : rest) {
            if (waves.empty() || (wave_bytes && ws + L.plans[i].state > wave_bytes)) {
                waves.emplace_back();
                ws = 0;
            }
            waves.back().push_back(i);
            ws += L.plans[i].state;
        }
    }
    add_groups(h, small, L, L.small);
    for (const std::vector<int> &w : waves) {
        // the instances of a wave share the caches
        uint64_t state = 0;
        for (int i : w) state += L.plans[i].state;
        BatchWave bw{(uint32_t)L.order.size(), (uint32_t)w.size(), 0, {}};
        for (int i : w) {
            L.plans[i].nt = stream_choice(state);
            bw.Kmax = std::max(bw.Kmax, L.plans[i].K);
        }
        add_groups(h, w, L, bw.groups);
        L.waves.push_back(std::move(bw));
    }
    L.tab_off = 0;
    L.map_off = align256((size_t)count * sizeof(Inst));
    L.inst_off = L.map_off + align256(L.map_words * 4 + 4);
    L.region_off.resize(count);
    size_t off = L.inst_off;
    for (int i = 0; i < count; ++i) {
        L.region_off[i] = off;
        off += instance_bytes(L.plans[i]);
    }
    L.total = off;
    return true;
}
}  // namespace

size_t kpm_workspace_bytes_batched(kpm_ham *const *h, int32_t count, const int32_t *M, const int32_t *R, int32_t vec)
{
    BatchLayout L;
    if (!batch_layout(h, count, M, R, vec, L)) return 0;
    return L.total;
}

kpm_status kpm_moments_batched(kpm_ham *const *h, int32_t count, const int32_t *M, const int32_t *R, int32_t vec,
                               const uint64_t *seed, const uint64_t *instance, void *ws, size_t ws_bytes,
                               double *const *mu_dev, void *stream)
{
    BatchLayout L;
    if (!seed || !instance || !mu_dev || !batch_layout(h, count, M, R, vec, L)) return KPM_ERR_INVALID_ARG;
    for (int i = 0; i < count; ++i)
        if (!mu_dev[i]) return KPM_ERR_INVALID_ARG;
    if (!ws || ((uintptr_t)ws & 255) || ws_bytes < L.total) return KPM_ERR_WORKSPACE;
    if (ensure_phase_table() != KPM_OK) return KPM_ERR_DEVICE;
    hipStream_t st = S(stream);
    char *base = (char *)ws;
    std::vector<Inst> tab(count);
    int32_t Mmax = 0;
    for (int t = 0; t < count; ++t) {
        const int i = L.order[t];
        fill_inst(h[i], L.plans[i], M[i], R[i], vec, seed[i], instance[i], base + L.region_off[i], tab[t]);
        tab[t].mu = mu_dev[i];
        Mmax = std::max(Mmax, M[i]);
    }
    // block maps, with the placement batch_layout sized them for
    std::vector<uint32_t> map;
    std::vector<const BatchGroup *> all;
    for (const BatchWave &w : L.waves)
        for (const BatchGroup &g : w.groups) all.push_back(&g);
    for (const BatchGroup *g : all) {
        std::vector<Inst> ins(tab.begin() + g->first, tab.begin() + g->first + g->count);
        if (map.size() != g->map_off || place_blocks(ins, map, true) != g->blocks) return KPM_ERR_INVALID_ARG;
        std::copy(ins.begin(), ins.end(), tab.begin() + g->first);
    }
    Inst *tab_dev = (Inst *)(base + L.tab_off);
    uint32_t *map_dev = (uint32_t *)(base + L.map_off);
    kpm_status e = upload(tab_dev, tab.data(), tab.size() * sizeof(Inst), st);
    if (e == KPM_OK && !map.empty()) e = upload(map_dev, map.data(), map.size() * 4, st);
    for (const BatchGroup &g : L.small) {
        int32_t kmax = 0;
        for (uint32_t t = g.first; t < g.first + g.count; ++t) kmax = std::max(kmax, L.plans[L.order[t]].K);
        if (e == KPM_OK) e = launch_small(L.prec, g.opk, tab_dev + g.first, g.count, g.lds, st);
        if (e == KPM_OK) e = launch_reduce(tab_dev + g.first, (int32_t)g.count, -1, kmax + 1, st);
    }
    for (const BatchWave &w : L.waves) {
        for (const BatchGroup &g : w.groups)
            if (e == KPM_OK) e = launch_init(L.prec, g.wide, tab_dev + g.first, map_dev + g.map_off, g.blocks, st);
        Inst *wt = tab_dev + w.first;
        int32_t written = 1, reduced = 0;  // dots indices, in lockstep for every instance of the wave
        for (int32_t k = 0; k < w.Kmax && e == KPM_OK; ++k) {
            if (written - reduced >= PSLOTS_MAX) {
                e = launch_reduce(wt, (int32_t)w.count, reduced - 1, written - reduced, st);
                reduced = written;
            }
            for (const BatchGroup &g : w.groups)
                if (e == KPM_OK)
                    e = launch_step(L.prec, g.opk, g.mode, g.wide, g.nt, tab_dev + g.first, map_dev + g.map_off,
                                    g.blocks, k, st);
            written += 1;
        }
        if (e == KPM_OK) e = launch_reduce(wt, (int32_t)w.count, reduced - 1, written - reduced, st);
    }
    if (e == KPM_OK) e = launch_moments(tab_dev, count, Mmax, st);
    return e;
}

// ---------------------------------------------------------------------------
// dynamic batches: begun solves advanced together, each at its own step
// ---------------------------------------------------------------------------
struct kpm_batch {
    int32_t capacity;
    char *mem;
    size_t map_words;
    std::vector<kpm_solve *> members;
};

kpm_status kpm_batch_create(int32_t capacity, kpm_batch **out)
{
    if (!out || capacity < 1 || capacity > 65535) return KPM_ERR_INVALID_ARG;
    kpm_batch *b = new (std::nothrow) kpm_batch();
    if (!b) return KPM_ERR_OUT_OF_MEMORY;
    b->capacity = capacity;
    b->map_words = (size_t)(std::min(capacity, 64) + 8) * 2048;
    const size_t bytes = align256((size_t)capacity * sizeof(Inst)) + b->map_words * 4;
    if (hipMalloc((void **)&b->mem, bytes) != hipSuccess) {
        delete b;
        return KPM_ERR_OUT_OF_MEMORY;
    }
    *out = b;
    return KPM_OK;
}

namespace {
// Grow the batch's table + block-map memory to hold `words` map entries.  The
// old memory may still be read by launches in flight on `st`, so wait for them.
kpm_status batch_reserve(kpm_batch *b, size_t words, hipStream_t st)
{
    if (words <= b->map_words) return KPM_OK;
    if (hipStreamSynchronize(st) != hipSuccess) return KPM_ERR_DEVICE;
    const size_t nw = std::max(words, 2 * b->map_words);
    char *mem = nullptr;
    if (hipMalloc((void **)&mem, align256((size_t)b->capacity * sizeof(Inst)) + nw * 4) != hipSuccess)
        return KPM_ERR_OUT_OF_MEMORY;
    if (hipFree(b->mem) != hipSuccess) {
        (void)hipFree(mem);
        return KPM_ERR_DEVICE;
    }
    b->mem = mem;
    b->map_words = nw;
    return KPM_OK;
}
}  // namespace

void kpm_batch_free(kpm_batch *b)
{
    if (!b) return;
    if (b->mem) (void)hipFree(b->mem);
    delete b;
}

kpm_status kpm_batch_add(kpm_batch *b, kpm_solve *s)
{
    if (!b || !s) return KPM_ERR_INVALID_ARG;
    if (std::find(b->members.begin(), b->members.end(), s) != b->members.end()) return KPM_ERR_INVALID_ARG;
    if ((int32_t)b->members.size() >= b->capacity) return KPM_ERR_UNSUPPORTED;
    if (!b->members.empty() && b->members[0]->h->prec != s->h->prec) return KPM_ERR_INVALID_ARG;
    b->members.push_back(s);
    return KPM_OK;
}

kpm_status kpm_batch_remove(kpm_batch *b, kpm_solve *s)
{
    if (!b || !s) return KPM_ERR_INVALID_ARG;
    auto it = std::find(b->members.begin(), b->members.end(), s);
    if (it == b->members.end()) return KPM_ERR_INVALID_ARG;
    b->members.erase(it);
    return KPM_OK;
}

int32_t kpm_batch_size(const kpm_batch *b) { return b ? (int32_t)b->members.size() : -1; }

kpm_status kpm_solve_remaining(const kpm_solve *s, int32_t *remaining)
{
    if (!s || !remaining) return KPM_ERR_INVALID_ARG;
    *remaining = s->inst.K - s->next;
    return KPM_OK;
}

kpm_status kpm_batch_advance(kpm_batch *b, int32_t steps, void *stream)
{
    if (!b || steps < 0) return KPM_ERR_INVALID_ARG;
    hipStream_t st = S(stream);
    steps = std::min(steps, PSLOTS_MAX);   // after the reductions below every ring has room for PSLOTS_MAX
    // active members grouped by kernel class; the table also carries each
    // member's pending reduction range
    std::vector<kpm_solve *> act;
    for (kpm_solve *s : b->members)
        if (s->inst.mode != MODE_SMALL && (s->next < s->inst.K || s->written > s->reduced)) act.push_back(s);
    if (act.empty() || steps == 0) return KPM_OK;
    // the members of one launch share the caches
    uint64_t state = 0;
    for (kpm_solve *s : act) state += s->state;
    const int nt = stream_choice(state);
    // one-step members by kernel class; temporally blocked members by (hopping,
    // addressing, depth of their full passes)
    auto key_of = [&](const kpm_solve *s) {
        if (s->inst.mode == MODE_TB) return 1000 + (s->inst.opk * 2 + s->wide) * 8 + s->inst.tbh;
        if (s->inst.mode == MODE_TB3) return 2000 + s->inst.opk * 2 + s->wide;
        return kernel_key(s->inst.opk, s->inst.mode, s->wide, nt);
    };
    std::vector<int> keys;
    for (kpm_solve *s : act) {
        const int key = key_of(s);
        if (std::find(keys.begin(), keys.end(), key) == keys.end()) keys.push_back(key);
    }
    std::vector<Inst> tab;
    std::vector<uint32_t> map;
    struct Group {
        int opk, mode, wide, nt;
        uint32_t first, count, blocks;
        size_t map_off;
        int tbh, maxfull;   // blocked groups: depth of the full passes, most full passes of a member
        uint32_t rems;      // blocked groups: bit r set if a member ends the chunk with a pass of depth r
    };
    std::vector<Group> groups;
    int32_t max_red = 0;
    for (int key : keys) {
        Group g{0, 0, 0, 0, (uint32_t)tab.size(), 0, 0, map.size(), 0, 0, 0u};
        std::vector<Inst> ins;
        for (kpm_solve *s : act) {
            if (key_of(s) != key) continue;
            Inst I = s->inst;
            I.nt = nt;
            I.step0 = s->next;
            I.red_lo = s->reduced;
            I.red_n = s->written - s->reduced;
            max_red = std::max(max_red, I.red_n);
            if (I.mode == MODE_TB || I.mode == MODE_TB3) {
                const int32_t adv = std::min(steps, I.K - s->next);
                I.tbfull = adv / I.tbh;
                I.tbrem = adv % I.tbh;
                I.tbp = s->tb_prev;
                I.tbc = s->tb_cur;
                g.tbh = I.tbh;
                g.maxfull = std::max(g.maxfull, I.tbfull);
                if (I.tbrem) g.rems |= 1u << I.tbrem;
            }
            g.opk = I.opk;
            g.mode = I.mode;
            g.wide = s->wide;
            g.nt = I.nt;
            ins.push_back(I);
        }
        g.count = (uint32_t)ins.size();
        g.blocks = place_blocks(ins, map);
        tab.insert(tab.end(), ins.begin(), ins.end());
        groups.push_back(g);
    }
    if (kpm_status r = batch_reserve(b, map.size(), st)) return r;
    Inst *tab_dev = (Inst *)b->mem;
    uint32_t *map_dev = (uint32_t *)(b->mem + align256((size_t)b->capacity * sizeof(Inst)));
    kpm_status e = upload(tab_dev, tab.data(), tab.size() * sizeof(Inst), st);
    if (e == KPM_OK && !map.empty()) e = upload(map_dev, map.data(), map.size() * 4, st);
    if (e == KPM_OK && max_red > 0) {
        hipLaunchKernelGGL(k_reduce_ranges, dim3(max_red, (uint32_t)tab.size()), dim3(BLOCK), 0, st, tab_dev);
        e = check_launch();
    }
    const int prec = act[0]->h->prec;
    // step k of the one-step members; the blocked members' full passes start at
    // the steps k = j * tbh, their last, shorter passes follow the loop
    for (int32_t k = 0; k < steps && e == KPM_OK; ++k)
        for (const Group &g : groups) {
            if (e != KPM_OK) break;
            if (g.mode != MODE_TB && g.mode != MODE_TB3)
                e = launch_step(prec, g.opk, g.mode, g.wide, g.nt, tab_dev + g.first, map_dev + g.map_off, g.blocks, k,
                                st);
            else if (k % g.tbh == 0 && k / g.tbh < g.maxfull)
                e = launch_pass(g.mode, g.tbh, prec, g.opk, g.wide, g.nt, tab_dev + g.first, map_dev + g.map_off,
                                g.blocks, k / g.tbh, nullptr, nullptr, nullptr, nullptr, st);
        }
    for (const Group &g : groups)
        for (int r = 1; r < 7 && e == KPM_OK; ++r)
            if ((g.mode == MODE_TB || g.mode == MODE_TB3) && (g.rems >> r & 1u))
                e = launch_pass(g.mode, r, prec, g.opk, g.wide, g.nt, tab_dev + g.first, map_dev + g.map_off, g.blocks,
                                -1, nullptr, nullptr, nullptr, nullptr, st);
    if (e != KPM_OK) return e;
    for (kpm_solve *s : act) {
        s->reduced = s->written;
        const int32_t done = std::min(steps, s->inst.K - s->next);
        if (s->inst.mode == MODE_TB || s->inst.mode == MODE_TB3) {
            for (int32_t j = 0; j < done / s->inst.tbh; ++j) tb_rotate(s->tb_prev, s->tb_cur, s->inst.tbh);
            if (done % s->inst.tbh) tb_rotate(s->tb_prev, s->tb_cur, done % s->inst.tbh);
        }
        s->next += done;
        s->written += done;
    }
    return KPM_OK;
}

// ---------------------------------------------------------------------------
// captured graphs of a whole batched solve
// ---------------------------------------------------------------------------
struct kpm_graph {
    hipGraph_t graph;
    hipGraphExec_t exec;
};

kpm_status kpm_graph_capture_batched(kpm_ham *const *h, int32_t count, const int32_t *M, const int32_t *R,
                                     int32_t vec, const uint64_t *seed, const uint64_t *instance, void *ws,
                                     size_t ws_bytes, double *const *mu_dev, void *stream, kpm_graph **out)
{
    if (!out || !stream) return KPM_ERR_INVALID_ARG;      // capture needs a non-default stream
    hipStream_t st = S(stream);
    if (ensure_phase_table() != KPM_OK) return KPM_ERR_DEVICE;
    // set LDS limits of the small-solve kernels outside the capture
    for (int i = 0; i < count; ++i) {
        Plan p;
        if (h && h[i] && M && R && make_plan(h[i], M[i], R[i], vec, p, false) && p.mode == MODE_SMALL) {
            small_fn f = h[i]->prec == KPM_F64 ? small_for<double>(h[i]->opk) : small_for<float>(h[i]->opk);
            if (hipFuncSetAttribute((const void *)f, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)small_lds_limit()) != hipSuccess)
                return KPM_ERR_DEVICE;
        }
    }
    if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) return KPM_ERR_DEVICE;
    kpm_status e = kpm_moments_batched(h, count, M, R, vec, seed, instance, ws, ws_bytes, mu_dev, stream);
    hipGraph_t g = nullptr;
    hipError_t ce = hipStreamEndCapture(st, &g);
    if (e != KPM_OK) {
        if (g) (void)hipGraphDestroy(g);
        return e;
    }
    if (ce != hipSuccess || !g) return KPM_ERR_DEVICE;
    hipGraphExec_t x = nullptr;
    if (hipGraphInstantiate(&x, g, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(g);
        return KPM_ERR_DEVICE;
    }
    kpm_graph *G = new (std::nothrow) kpm_graph();
    if (!G) {
        (void)hipGraphExecDestroy(x);
        (void)hipGraphDestroy(g);
        return KPM_ERR_OUT_OF_MEMORY;
    }
    G->graph = g;
    G->exec = x;
    *out = G;
    return KPM_OK;
}

kpm_status kpm_graph_launch(kpm_graph *g, void *stream)
{
    if (!g) return KPM_ERR_INVALID_ARG;
    return hipGraphLaunch(g->exec, S(stream)) == hipSuccess ? KPM_OK : KPM_ERR_DEVICE;
}

void kpm_graph_free(kpm_graph *g)
{
    if (!g) return;
    (void)hipGraphExecDestroy(g->exec);
    (void)hipGraphDestroy(g->graph);
    delete g;
}

// ---------------------------------------------------------------------------
// Lanczos spectral interval
// ---------------------------------------------------------------------------
extern "C++" {
namespace {
typedef void (*lz_matvec_fn)(const Inst *, const void *, void *, int32_t);
template <bool WIDE>
lz_matvec_fn lz_matvec_for(int opk)
{
    switch (opk) {
    case OP_REAL2: return k_lz_matvec<OP_REAL2, WIDE>;
    case OP_REAL3: return k_lz_matvec<OP_REAL3, WIDE>;
    case OP_SPIN2: return k_lz_matvec<OP_SPIN2, WIDE>;
    case OP_SPIN3: return k_lz_matvec<OP_SPIN3, WIDE>;
    case OP_CSR_R: return k_lz_matvec<OP_CSR_R, WIDE>;
    default: return k_lz_matvec<OP_CSR_C, WIDE>;
    }
}

// One FP64 vector (R = 1) in the flat layout; dots indices 0 .. 2k + 2.
bool lanczos_plan(const kpm_ham *h, int32_t k, Plan &p, int32_t &vec)
{
    if (!h || h->prec != KPM_F64 || k < 1 || k > LZ_KMAX) return false;
    vec = h->cplx_op ? KPM_VEC_PHASE : KPM_VEC_RADEMACHER;
    if (!make_plan(h, 2, 1, vec, p, false)) return false;
    p.mode = MODE_FLAT;
    const uint64_t per_tile = (uint64_t)BLOCK * p.tpt;
    p.tiles = (uint32_t)((p.nel + per_tile - 1) / per_tile);
    p.xcd = p.tiles >= XCD_MIN_ITEMS ? 1 : 0;
    p.nb = std::min<uint32_t>((p.tiles + 7) / 8 * 8, (uint32_t)g_max_blocks);
    p.K = 2 * k + 2;
    p.P_slots = 2;
    p.part_bytes = align256((size_t)p.P_slots * p.tiles * 4 * sizeof(double));
    p.dots_bytes = align256((size_t)(p.K + 1) * 4 * sizeof(double));
    p.buf_bytes = align256((size_t)h->N * p.Rs * p.esz);
    return true;
}
}  // namespace
}  // extern "C++"

size_t kpm_lanczos_workspace_bytes(const kpm_ham *h, int32_t k)
{
    Plan p;
    int32_t vec;
    if (!lanczos_plan(h, k, p, vec)) return 0;
    return align256(sizeof(Inst)) + p.part_bytes + p.dots_bytes + 3 * p.buf_bytes;
}

kpm_status kpm_bounds_lanczos(kpm_ham *h, int32_t k, uint64_t seed, double pad, double clamp_lo, double clamp_hi,
                              void *ws, size_t ws_bytes, double *out_dev, void *stream)
{
    if (!h || !out_dev || k < 1 || k > LZ_KMAX || !(pad >= 0.0) || !std::isfinite(pad) || std::isnan(clamp_lo) ||
        std::isnan(clamp_hi) || !(clamp_lo < clamp_hi))
        return KPM_ERR_INVALID_ARG;
    if (h->prec != KPM_F64) return KPM_ERR_UNSUPPORTED;
    Plan p;
    int32_t vec;
    if (!lanczos_plan(h, k, p, vec)) return KPM_ERR_INVALID_ARG;
    if (!ws || ((uintptr_t)ws & 255) || ws_bytes < kpm_lanczos_workspace_bytes(h, k)) return KPM_ERR_WORKSPACE;
    if (ensure_phase_table() != KPM_OK) return KPM_ERR_DEVICE;
    hipStream_t st = S(stream);
    char *base = (char *)ws;
    Inst I;
    fill_inst(h, p, 2, 1, vec, seed, 0, base + align256(sizeof(Inst)), I);
    void *vb[2] = {I.buf0, I.buf1};
    void *ub = (char *)I.buf1 + p.buf_bytes;
    Inst *tab = (Inst *)base;
    const bool wide = p.wide != 0;
    const lz_matvec_fn mv = wide ? lz_matvec_for<true>(h->opk) : lz_matvec_for<false>(h->opk);
    auto update = wide ? k_lz_update<true> : k_lz_update<false>;
    auto scale = wide ? k_lz_scale<true> : k_lz_scale<false>;
    const dim3 grid(p.nb), blk(BLOCK);
    kpm_status e = upload(tab, &I, sizeof(Inst), st);
    if (e == KPM_OK) e = launch_init(KPM_F64, p.wide, tab, nullptr, p.nb, st);       // xi, <xi|xi> partials
    if (e == KPM_OK) e = launch_reduce(tab, 1, -1, 1, st);                          // dots[0]
    if (e == KPM_OK) {
        hipLaunchKernelGGL(scale, grid, blk, 0, st, tab, vb[0], 0);                  // v_0
        e = check_launch();
    }
    int cur = 0;
    for (int32_t j = 0; j < k && e == KPM_OK; ++j) {
        hipLaunchKernelGGL(mv, grid, blk, 0, st, tab, (const void *)vb[cur], ub, 2 * j + 1);
        e = check_launch();
        if (e == KPM_OK) e = launch_reduce(tab, 1, 2 * j, 1, st);
        if (e == KPM_OK) {
            hipLaunchKernelGGL(update, grid, blk, 0, st, tab, (const void *)ub, (const void *)vb[cur], vb[cur ^ 1], j);
            e = check_launch();
        }
        if (e == KPM_OK) e = launch_reduce(tab, 1, 2 * j + 1, 1, st);
        if (e == KPM_OK) {
            hipLaunchKernelGGL(scale, grid, blk, 0, st, tab, vb[cur ^ 1], 2 * j + 2);
            e = check_launch();
        }
        cur ^= 1;
    }
    if (e == KPM_OK) {
        hipLaunchKernelGGL(k_lz_tridiag, dim3(1), dim3(64), 0, st, tab, k, pad, h->a, h->b, clamp_lo, clamp_hi,
                           out_dev);
        e = check_launch();
    }
    return e;
}

// ---------------------------------------------------------------------------
// dense-H recursion
// ---------------------------------------------------------------------------
extern "C++" {
namespace {
constexpr int64_t DENSE_RESIDENT_MAX = 128;   // H~ (FP64) and one vector slab fit one CU's LDS
struct DenseLayout {
    bool resident;
    uint32_t tn;           // output columns per block of the tiled kernel (64 or 32)
    uint32_t Dp, Rp, blocks, tiles;   // grid; partial sums per step (resident: one per wave)
    int32_t K, P_slots;
    size_t ht_off, v0_off, v1_off, part_off, dots_off, total;
};
bool dense_layout(int64_t D, int32_t M, int32_t R, DenseLayout &L)
{
    if (D < 1 || D > 65536 || M < 1 || R < 1 || R > (1 << 20)) return false;
    // the on-chip path keeps every step's per-wave dot partials until the end:
    // (M/2 + 1) x (R/16 slabs) x (D/16 waves) x 32 bytes, held to 256 MiB
    const uint64_t res_part = ((uint64_t)(M / 2) + 1) * (uint64_t)((R + 15) / 16) * (uint64_t)((D + 15) / 16) * 32;
    L.resident = g_small && D <= DENSE_RESIDENT_MAX && res_part <= (256ull << 20);
    const uint32_t q = L.resident ? 16 : DN_TILE;
    L.Dp = (uint32_t)((D + q - 1) / q * q);
    L.Rp = (uint32_t)((R + q - 1) / q * q);
    if ((uint64_t)L.Dp * L.Rp >= (1ull << 40)) return false;
    // 64 x 64 output blocks, or 64 x 32 when that leaves fewer than 4 blocks per CU
    L.tn = ((L.Dp / DN_TILE) * (L.Rp / DN_TILE) < 1024) ? 32 : DN_TILE;
    L.blocks = L.resident ? L.Rp / 16 : (L.Dp / DN_TILE) * (L.Rp / L.tn);
    L.tiles = L.resident ? L.blocks * (L.Dp / 16) : L.blocks;
    L.K = M / 2;
    L.P_slots = L.resident ? L.K + 1 : std::min(L.K + 1, PSLOTS_MAX);
    const size_t vbytes = L.resident ? 0 : align256((size_t)L.Dp * L.Rp * 8);
    L.ht_off = align256(sizeof(Inst));
    L.v0_off = L.ht_off + align256((size_t)L.Dp * L.Dp * 8);
    L.v1_off = L.v0_off + vbytes;
    L.part_off = L.v1_off + vbytes;
    L.dots_off = L.part_off + align256((size_t)L.P_slots * L.tiles * 4 * 8);
    L.total = L.dots_off + align256((size_t)(L.K + 1) * 4 * 8);
    return true;
}
}  // namespace
}  // extern "C++"

size_t kpm_dense_workspace_bytes(int64_t D, int32_t M, int32_t R)
{
    DenseLayout L;
    return dense_layout(D, M, R, L) ? L.total : 0;
}

kpm_status kpm_dense_moments(const double *H_dev, int64_t D, double a, double b, int32_t M, int32_t R, int32_t vec,
                             uint64_t seed, uint64_t instance, void *ws, size_t ws_bytes, double *mu_dev, void *stream)
{
    DenseLayout L;
    if (!H_dev || !mu_dev || !(a > 0.0) || !std::isfinite(b) || !dense_layout(D, M, R, L)) return KPM_ERR_INVALID_ARG;
    if (vec != KPM_VEC_RADEMACHER && vec != KPM_VEC_UNIT) return KPM_ERR_UNSUPPORTED;   // real vectors only
    if (!ws || ((uintptr_t)ws & 255) || ws_bytes < L.total) return KPM_ERR_WORKSPACE;
    if (ensure_phase_table() != KPM_OK) return KPM_ERR_DEVICE;
    hipStream_t st = S(stream);
    char *base = (char *)ws;
    double *Ht = (double *)(base + L.ht_off);
    double *V[2] = {(double *)(base + L.v0_off), (double *)(base + L.v1_off)};
    double *part = (double *)(base + L.part_off);
    Inst I;
    std::memset(&I, 0, sizeof(I));
    I.mode = MODE_FLAT;
    I.tiles = L.tiles;
    I.pslots = L.P_slots;
    I.K = L.K;
    I.M = M;
    I.R = R;
    I.vec = vec;
    I.norm = (vec == KPM_VEC_UNIT) ? (double)R : (double)D * (double)R;
    I.partial = part;
    I.dots = (double *)(base + L.dots_off);
    I.mu = mu_dev;
    Inst *tab = (Inst *)base;
    kpm_status e = upload(tab, &I, sizeof(Inst), st);
    if (e == KPM_OK) {
        const uint64_t n2 = (uint64_t)L.Dp * L.Dp;
        hipLaunchKernelGGL(k_dense_scale, dim3((uint32_t)((n2 + 255) / 256)), dim3(256), 0, st, H_dev, (uint32_t)D, L.Dp,
                           a, b, Ht);
        e = check_launch();
    }
    if (e == KPM_OK && L.resident) {
        typedef void (*res_fn)(const double *, uint32_t, uint32_t, int, uint64_t, uint64_t, int32_t, double *);
        static const res_fn fns[8] = {k_dense_resident<1>, k_dense_resident<2>, k_dense_resident<3>,
                                      k_dense_resident<4>, k_dense_resident<5>, k_dense_resident<6>,
                                      k_dense_resident<7>, k_dense_resident<8>};
        const int nw = (int)(L.Dp / 16);
        const size_t lds = (size_t)L.Dp * 16 * 8;
        if (hipFuncSetAttribute((const void *)fns[nw - 1], hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) !=
            hipSuccess)
            return KPM_ERR_DEVICE;
        hipLaunchKernelGGL(fns[nw - 1], dim3(L.blocks), dim3(64 * nw), lds, st, Ht, (uint32_t)D, (uint32_t)R, vec, seed,
                           instance, L.K, part);
        e = check_launch();
        if (e == KPM_OK) e = launch_reduce(tab, 1, -1, L.K + 1, st);
        if (e == KPM_OK) e = launch_moments(tab, 1, M, st);
        return e;
    }
    if (e == KPM_OK) {
        hipLaunchKernelGGL(k_dense_init, dim3(L.tiles), dim3(256), 0, st, (uint32_t)D, L.Dp, (uint32_t)R, L.Rp, vec, seed,
                           instance, L.tn, V[0], part);
        e = check_launch();
    }
    int32_t written = 1, reduced = 0;
    for (int32_t n = 0; n < L.K && e == KPM_OK; ++n) {
        if (written - reduced >= L.P_slots) {
            e = launch_reduce(tab, 1, reduced - 1, written - reduced, st);
            reduced = written;
            if (e != KPM_OK) break;
        }
        double *pslot = part + (size_t)((n + 1) % L.P_slots) * L.tiles * 4;
        typedef void (*step_fn)(const double *, const double *, double *, uint32_t, uint32_t, double *);
        const step_fn f = L.tn == 32 ? (n == 0 ? k_dense_step<true, 32> : k_dense_step<false, 32>)
                                     : (n == 0 ? k_dense_step<true, 64> : k_dense_step<false, 64>);
        hipLaunchKernelGGL(f, dim3(L.tiles), dim3(256), 0, st, Ht, V[n & 1], V[(n + 1) & 1], L.Dp, L.Rp, pslot);
        e = check_launch();
        written += 1;
    }
    if (e == KPM_OK) e = launch_reduce(tab, 1, reduced - 1, written - reduced, st);
    if (e == KPM_OK) e = launch_moments(tab, 1, M, st);
    return e;
}

kpm_status kpm_dos(const double *mu_dev, int32_t M, int32_t jackson, int32_t K, double a, double b, double *omega_dev,
                   double *rho_dev, void *stream)
{
    if (!mu_dev || !omega_dev || !rho_dev || M < 1 || K < 1 || !(a > 0.0) || !std::isfinite(b)) return KPM_ERR_INVALID_ARG;
    hipLaunchKernelGGL(k_dos, dim3((K + DOS_PTS - 1) / DOS_PTS), dim3(256), 0, S(stream), mu_dev, M, jackson ? 1 : 0, K, a, b,
                       omega_dev, rho_dev);
    return check_launch();
}

kpm_status kpm_green(const double *mu_dev, int32_t M, int32_t kernel, double lambda, int32_t K, double a, double b,
                     double *omega_dev, double *g_re_dev, double *g_im_dev, void *stream)
{
    if (!mu_dev || !omega_dev || !g_re_dev || !g_im_dev || M < 1 || K < 1 || kernel < 0 || kernel > 2 ||
        !(a > 0.0) || !std::isfinite(b) || (kernel == 2 && !(lambda > 0.0 && lambda < 700.0)))
        return KPM_ERR_INVALID_ARG;
    hipLaunchKernelGGL(k_green, dim3((K + DOS_PTS - 1) / DOS_PTS), dim3(256), 0, S(stream), mu_dev, M, kernel, lambda, K, a, b,
                       omega_dev, g_re_dev, g_im_dev);
    return check_launch();
}

kpm_status kpm_start_vectors(int32_t vec, int32_t complex_layout, uint64_t seed, uint64_t instance, int64_t N, int32_t R,
                             double *out_dev, void *stream)
{
    if (!out_dev || vec < 0 || vec > 2 || N < 1 || R < 1 || N >= (1ll << 31) || (double)N * R >= 4.0e9)
        return KPM_ERR_INVALID_ARG;
    const uint64_t n = (uint64_t)N * R;
    const int cplx = (complex_layout || vec == KPM_VEC_PHASE) ? 1 : 0;
    if (ensure_phase_table() != KPM_OK) return KPM_ERR_DEVICE;
    hipLaunchKernelGGL(k_export_start, dim3((uint32_t)((n + 255) / 256)), dim3(256), 0, S(stream), vec, cplx, seed,
                       instance, (uint32_t)N, (uint32_t)R, out_dev);
    return check_launch();
}

kpm_status kpm_set_launch(int32_t key, int32_t value)
{
    switch (key) {
    case KPM_LAUNCH_ELEMS_PER_THREAD:
        if (value != 1 && value != 2 && value != 4) return KPM_ERR_INVALID_ARG;
        g_tpt = value;
        return KPM_OK;
    case KPM_LAUNCH_MAX_BLOCKS:
        if (value < 8 || (value % 8) != 0) return KPM_ERR_INVALID_ARG;
        g_max_blocks = value;
        return KPM_OK;
    case KPM_LAUNCH_MARCH:
        if (value != 0 && value != 1) return KPM_ERR_INVALID_ARG;
        g_march = value;
        return KPM_OK;
    case KPM_LAUNCH_MARCH_ITEMS:
        if (value < 1) return KPM_ERR_INVALID_ARG;
        g_march_items = value;
        return KPM_OK;
    case KPM_LAUNCH_XCD_SPLIT:
        if (value < 0 || value > 3) return KPM_ERR_INVALID_ARG;
        g_xcd_split = value;
        return KPM_OK;
    case KPM_LAUNCH_ALTERNATE:
        if (value != 0 && value != 1) return KPM_ERR_INVALID_ARG;
        g_alternate = value;
        return KPM_OK;
    case KPM_LAUNCH_SMALL:
        if (value != 0 && value != 1) return KPM_ERR_INVALID_ARG;
        g_small = value;
        return KPM_OK;
    case KPM_LAUNCH_STREAMING:
        if (value < 0 || value > 2) return KPM_ERR_INVALID_ARG;
        g_streaming = value;
        return KPM_OK;
    case KPM_LAUNCH_WAVE_MIB:
        if (value < 0 || value > (1 << 22)) return KPM_ERR_INVALID_ARG;
        g_wave_mib = value;
        return KPM_OK;
    case KPM_LAUNCH_TBLOCK:
        if (value < -1 || value == 2 || value > 6) return KPM_ERR_INVALID_ARG;
        g_tblock = value;
        return KPM_OK;
    case KPM_LAUNCH_TB3:
        if (value < -1 || value > 1) return KPM_ERR_INVALID_ARG;
        g_tb3 = value;
        return KPM_OK;
    case KPM_LAUNCH_TB_GROUP:
        if (value < 0 || value > 512) return KPM_ERR_INVALID_ARG;
        g_tb_group = value;
        return KPM_OK;
    }
    return KPM_ERR_INVALID_ARG;
}

kpm_status kpm_get_launch(int32_t key, int32_t *value)
{
    if (!value) return KPM_ERR_INVALID_ARG;
    switch (key) {
    case KPM_LAUNCH_ELEMS_PER_THREAD: *value = g_tpt; return KPM_OK;
    case KPM_LAUNCH_MAX_BLOCKS: *value = g_max_blocks; return KPM_OK;
    case KPM_LAUNCH_MARCH: *value = g_march; return KPM_OK;
    case KPM_LAUNCH_MARCH_ITEMS: *value = g_march_items; return KPM_OK;
    case KPM_LAUNCH_XCD_SPLIT: *value = g_xcd_split; return KPM_OK;
    case KPM_LAUNCH_ALTERNATE: *value = g_alternate; return KPM_OK;
    case KPM_LAUNCH_SMALL: *value = g_small; return KPM_OK;
    case KPM_LAUNCH_STREAMING: *value = g_streaming; return KPM_OK;
    case KPM_LAUNCH_WAVE_MIB: *value = g_wave_mib; return KPM_OK;
    case KPM_LAUNCH_TBLOCK: *value = g_tblock; return KPM_OK;
    case KPM_LAUNCH_TB3: *value = g_tb3; return KPM_OK;
    case KPM_LAUNCH_TB_GROUP: *value = g_tb_group; return KPM_OK;
    }
    return KPM_ERR_INVALID_ARG;
}

// Host-side self-check of the division-by-constant helper (used by CPU tests).
int32_t kpm_selftest_fastdiv(uint32_t d, const uint32_t *n, int32_t count)
{
    if (d == 0) return -1;
    FastDiv f = make_fastdiv(d);
    for (int32_t k = 0; k < count; ++k)
        if (fdiv(n[k], f) != n[k] / d) return k + 1;
    return 0;
}

// Host check of the block placement of one launch group: nb[i] blocks, the
// XCD split flag xcd[i] (updated: 1 for instances the placement split, 0 for
// those it placed whole) and, optionally, units[i] work units of instance i
// (NULL: none).  wave = 0: flat instances of a dynamic batch; 1: march
// instances of a static batch wave.  Writes block0/bstride per instance and the
// per-block map (up to map_cap entries); returns the grid size, or -1 if the
// map does not fit.
int64_t kpm_selftest_placement(const uint32_t *nb, int32_t *xcd, const uint32_t *units, int32_t count, int32_t wave,
                               uint32_t *block0, uint32_t *bstride, uint32_t *map_out, int64_t map_cap)
{
    if (!nb || !xcd || count < 1 || !block0 || !bstride || !map_out) return -1;
    std::vector<Inst> ins(count);
    for (int32_t i = 0; i < count; ++i) {
        std::memset(&ins[i], 0, sizeof(Inst));
        ins[i].nb = nb[i];
        ins[i].xcd = xcd[i];
        ins[i].mode = wave ? MODE_MARCH : MODE_FLAT;
        ins[i].tiles = units ? units[i] : 0;
        ins[i].nct = units ? units[i] : 0;
    }
    std::vector<uint32_t> map;
    const uint32_t blocks = place_blocks(ins, map, wave != 0);
    if ((int64_t)map.size() > map_cap || map.size() != blocks) return -1;
    for (int32_t i = 0; i < count; ++i) {
        block0[i] = ins[i].block0;
        bstride[i] = ins[i].bstride;
        xcd[i] = ins[i].xcd;
    }
    std::copy(map.begin(), map.end(), map_out);
    return blocks;
}

}  // extern "C"
