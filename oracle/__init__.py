"""Plain FP64 CPU oracle for the Kernel Polynomial Method (KPM) moments and DoS.

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  Nothing here imports, loads or calls
the HIP library, and the HIP library shares no code with it.

Moments (Sec. II-A of Zhang, Yamagiwa, Okumura, Yunoki 2011): the C library
``libkpm_oracle.so`` (built from ``kpm_oracle.c``) evaluates the stochastic
trace estimator of Eq. (munr) by the vector recursion of Eq. (rn), once
directly ("formula A") and once through the product identity
T_m T_n = (T_{m+n} + T_{|m-n|})/2 ("formula B", two moments per product).

DoS (Eq. (fKPM) with the Jackson kernel named in Sec. I): written out below in
numpy from the definition: f(x) = [g_0 mu_0 + 2 sum_n g_n mu_n T_n(x)] /
(pi sqrt(1-x^2)) on the Chebyshev points x_k = cos(pi (k+1/2)/K), mapped
back to omega = a x + b with rho(omega) = f(x)/a (the change of variables
below Eq. (DoStr)).

Parity pins: every function here is checked, in tests/test_oracle_*.py,
against something other than itself (numpy's Philox, dense eigendecomposition,
closed-form lattice spectra, exact rational sums, invariants).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "kpm_oracle.c")
_LIB = os.path.join(_HERE, "libkpm_oracle.so")

VEC_RADEMACHER, VEC_PHASE, VEC_UNIT = 0, 1, 2
HOP_REAL, HOP_SPIN = 0, 1

_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain C99 + OpenMP, no fused multiply-add)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=gnu99", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
               "-shared", "-fPIC", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i64, u64, i32, f64 = ctypes.c_int64, ctypes.c_uint64, ctypes.c_int, ctypes.c_double
        lib.kpmo_philox4x64_10.argtypes = [P, P, P]
        lib.kpmo_philox4x64_10.restype = None
        lib.kpmo_start_vectors.argtypes = [i32, u64, u64, i64, i32, P, P]
        lib.kpmo_start_vectors.restype = None
        lib.kpmo_moments_lattice.argtypes = [i32, P, f64, i32, P, P, f64, f64, i32, i32, i32,
                                             u64, u64, i32, P, P, P]
        lib.kpmo_moments_lattice.restype = i32
        lib.kpmo_moments_csr.argtypes = [i64, P, P, P, P, f64, f64, i32, i32, i32,
                                         u64, u64, i32, P, P, P]
        lib.kpmo_moments_csr.restype = i32
        lib.kpmo_gershgorin_lattice.argtypes = [i32, P, f64, i32, P, P, P, P]
        lib.kpmo_gershgorin_lattice.restype = i32
        lib.kpmo_gershgorin_csr.argtypes = [i64, P, P, P, P, P, P]
        lib.kpmo_gershgorin_csr.restype = i32
        lib.kpmo_lanczos_lattice.argtypes = [i32, P, f64, i32, P, P, f64, f64, i32, i32, u64, u64, i32, P, P]
        lib.kpmo_lanczos_lattice.restype = i32
        lib.kpmo_lanczos_csr.argtypes = [i64, P, P, P, P, f64, f64, i32, i32, u64, u64, i32, P, P]
        lib.kpmo_lanczos_csr.restype = i32
        lib.kpmo_max_threads.argtypes = []
        lib.kpmo_max_threads.restype = i32
        _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def max_threads() -> int:
    return int(_load().kpmo_max_threads())


# --------------------------------------------------------------------------
# random numbers
# --------------------------------------------------------------------------
def philox4x64_10(counter, key):
    """One Philox4x64-10 block (Salmon et al., SC'11): 4 words from a 4-word counter and 2-word key."""
    c = np.ascontiguousarray(counter, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    _load().kpmo_philox4x64_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def start_vectors(vec_kind: int, seed: int, instance: int, N: int, R: int):
    """The random start vectors xi_{r,i} (Sec. II-A, stochastic trace), shape (R, N), complex128."""
    re = np.zeros((R, N))
    im = np.zeros((R, N))
    _load().kpmo_start_vectors(vec_kind, seed, instance, N, R, _ptr(re), _ptr(im))
    return re + 1j * im


# --------------------------------------------------------------------------
# spectral bounds and rescaling (Sec. II-A, Eq. (tilde))
# --------------------------------------------------------------------------
def gershgorin_lattice(dim, L, t, hop=HOP_REAL, onsite=None, spinor=None):
    Lv = np.ascontiguousarray(list(L) + [1] * (3 - len(L)), dtype=np.int64)
    lo = np.zeros(1)
    hi = np.zeros(1)
    st = _load().kpmo_gershgorin_lattice(dim, _ptr(Lv), float(t), hop, _ptr(_f64(onsite)),
                                         _ptr(_f64(spinor)), _ptr(lo), _ptr(hi))
    if st:
        raise ValueError(f"oracle gershgorin_lattice failed ({st})")
    return float(lo[0]), float(hi[0])


def gershgorin_csr(row_ptr, col, val_re, val_im=None):
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    cl = np.ascontiguousarray(col, dtype=np.int32)
    lo = np.zeros(1)
    hi = np.zeros(1)
    st = _load().kpmo_gershgorin_csr(len(rp) - 1, _ptr(rp), _ptr(cl), _ptr(_f64(val_re)),
                                     _ptr(_f64(val_im)), _ptr(lo), _ptr(hi))
    if st:
        raise ValueError(f"oracle gershgorin_csr failed ({st})")
    return float(lo[0]), float(hi[0])


def scale_from_bounds(e_lo: float, e_hi: float, eps: float = 0.01):
    """alpha_- and alpha_+ of Eq. (tilde) with a relative safety margin eps:
    a = (E_hi - E_lo) / (2 - eps), b = (E_hi + E_lo) / 2  (eps = 0 is the paper's literal choice)."""
    return (e_hi - e_lo) / (2.0 - eps), (e_hi + e_lo) / 2.0


# --------------------------------------------------------------------------
# Lanczos estimate of the spectral interval (an alternative to the Gershgorin
# bounds of Sec. II-A for the rescaling of Eq. (tilde))
# --------------------------------------------------------------------------
def lanczos_lattice(dim, L, t, a, b, k, vec_kind=VEC_RADEMACHER, seed=0, instance=0, hop=HOP_REAL,
                    onsite=None, spinor=None, nthreads=0):
    """Lanczos coefficients (alpha_0..alpha_{k-1}, beta_0..beta_{k-1}) of H~ = (H - b)/a on a
    periodic lattice, from start vector r = 0 of the given kind (the process in kpm_oracle.c)."""
    Lv = np.ascontiguousarray(list(L) + [1] * (3 - len(L)), dtype=np.int64)
    al = np.zeros(k)
    be = np.zeros(k)
    st = _load().kpmo_lanczos_lattice(dim, _ptr(Lv), float(t), hop, _ptr(_f64(onsite)), _ptr(_f64(spinor)),
                                      float(a), float(b), k, vec_kind, seed, instance, nthreads, _ptr(al),
                                      _ptr(be))
    if st:
        raise ValueError(f"oracle lanczos_lattice failed ({st})")
    return al, be


def lanczos_csr(row_ptr, col, val_re, val_im, a, b, k, vec_kind=VEC_RADEMACHER, seed=0, instance=0, nthreads=0):
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    cl = np.ascontiguousarray(col, dtype=np.int32)
    al = np.zeros(k)
    be = np.zeros(k)
    st = _load().kpmo_lanczos_csr(len(rp) - 1, _ptr(rp), _ptr(cl), _ptr(_f64(val_re)), _ptr(_f64(val_im)),
                                  float(a), float(b), k, vec_kind, seed, instance, nthreads, _ptr(al), _ptr(be))
    if st:
        raise ValueError(f"oracle lanczos_csr failed ({st})")
    return al, be


LANCZOS_BREAKDOWN = 1e-12


def lanczos_bounds(alpha, beta, a=1.0, b=0.0, pad=0.005, clamp=(-np.inf, np.inf)):
    """Spectral interval of H from the Lanczos coefficients of H~ = (H - b)/a.

    The process stops at the first j with beta_j <= 1e-12 max(|alpha|, |beta| up to j) (an
    invariant subspace), giving m = j + 1 coefficients; else m = k.  T is the m x m symmetric
    tridiagonal matrix with diagonal alpha_0..alpha_{m-1} and off-diagonal beta_0..beta_{m-2}.
    Its extreme eigenpairs (theta, y) come from a dense symmetric eigensolver; the residual bound
    of a Ritz pair is r = beta_{m-1} |y_{m-1}| (0 after a breakdown).  The interval of H~ is
    [theta_min - p_min, theta_max + p_max] with p = max(r, pad (theta_max - theta_min)), mapped to
    H by E = a lambda + b and clipped to `clamp` (an interval known to enclose the spectrum,
    e.g. the Gershgorin one).  Returns a dict with e_lo, e_hi, theta_min, theta_max, r_min, r_max, m."""
    alpha = np.asarray(alpha, dtype=np.float64)
    beta = np.asarray(beta, dtype=np.float64)
    k = len(alpha)
    m, scale, stop = k, 0.0, False
    for j in range(k):
        scale = max(scale, abs(alpha[j]), abs(beta[j]))
        if beta[j] <= LANCZOS_BREAKDOWN * scale:
            m, stop = j + 1, True
            break
    T = np.diag(alpha[:m]) + np.diag(beta[:m - 1], 1) + np.diag(beta[:m - 1], -1)
    w, V = np.linalg.eigh(T)
    blast = 0.0 if stop else beta[m - 1]
    th_lo, th_hi = float(w[0]), float(w[-1])
    r_lo, r_hi = blast * abs(V[m - 1, 0]), blast * abs(V[m - 1, -1])
    width = th_hi - th_lo
    lo = th_lo - max(r_lo, pad * width)
    hi = th_hi + max(r_hi, pad * width)
    e_lo = max(a * lo + b, clamp[0])
    e_hi = min(a * hi + b, clamp[1])
    return {"e_lo": e_lo, "e_hi": e_hi, "theta_min": th_lo, "theta_max": th_hi, "r_min": float(r_lo),
            "r_max": float(r_hi), "m": m}


# --------------------------------------------------------------------------
# moments
# --------------------------------------------------------------------------
def moments_lattice(dim, L, t, a, b, M, R, vec_kind=VEC_RADEMACHER, seed=0, instance=0,
                    hop=HOP_REAL, onsite=None, spinor=None, formula_a=False, nthreads=0,
                    return_dots=False):
    """Moments mu_0..mu_{M-1} on a periodic square (dim 2) or cubic (dim 3) lattice.

    Returns mu (formula B), and also mu_A (Eq. (munr) directly) when formula_a is set.
    """
    Lv = np.ascontiguousarray(list(L) + [1] * (3 - len(L)), dtype=np.int64)
    muB = np.zeros(M)
    muA = np.zeros(M) if formula_a else None
    K = M // 2
    dots = np.zeros((K + 1) * 4) if return_dots else None
    st = _load().kpmo_moments_lattice(dim, _ptr(Lv), float(t), hop, _ptr(_f64(onsite)),
                                      _ptr(_f64(spinor)), float(a), float(b), M, R, vec_kind,
                                      seed, instance, nthreads, _ptr(muB), _ptr(muA), _ptr(dots))
    if st:
        raise ValueError(f"oracle moments_lattice failed ({st})")
    out = [muB]
    if formula_a:
        out.append(muA)
    if return_dots:
        out.append(dots.reshape(K + 1, 2, 2))
    return out[0] if len(out) == 1 else tuple(out)


def moments_csr(row_ptr, col, val_re, val_im, a, b, M, R, vec_kind=VEC_RADEMACHER, seed=0,
                instance=0, formula_a=False, nthreads=0):
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    cl = np.ascontiguousarray(col, dtype=np.int32)
    muB = np.zeros(M)
    muA = np.zeros(M) if formula_a else None
    st = _load().kpmo_moments_csr(len(rp) - 1, _ptr(rp), _ptr(cl), _ptr(_f64(val_re)),
                                  _ptr(_f64(val_im)), float(a), float(b), M, R, vec_kind,
                                  seed, instance, nthreads, _ptr(muB), _ptr(muA), None)
    if st:
        raise ValueError(f"oracle moments_csr failed ({st})")
    return (muB, muA) if formula_a else muB


# --------------------------------------------------------------------------
# density of states, Eq. (fKPM)
# --------------------------------------------------------------------------
def jackson(M: int) -> np.ndarray:
    """Jackson kernel coefficients g_0..g_{M-1} for an M-moment expansion (the kernel the paper
    names in Sec. I; formula from the KPM literature it cites):
    g_n = [(M - n + 1) cos(pi n/(M+1)) + sin(pi n/(M+1)) cot(pi/(M+1))] / (M + 1)."""
    n = np.arange(M, dtype=np.float64)
    q = np.pi / (M + 1)
    return ((M - n + 1) * np.cos(q * n) + np.sin(q * n) / np.tan(q)) / (M + 1)


def chebyshev_points(K: int):
    """theta_k = pi (k + 1/2)/K and x_k = cos(theta_k), k = 0..K-1 (first-kind Chebyshev points)."""
    theta = np.pi * (np.arange(K) + 0.5) / K
    return theta, np.cos(theta)


def dos(mu, K: int, a: float, b: float, use_jackson: bool = True):
    """Eq. (fKPM) evaluated at the K Chebyshev points, returned as (omega, rho(omega)).

    cos(n theta_k) is evaluated as cos(pi m / (2K)) with m = n (2k+1) mod 4K, an exact integer
    reduction of the angle n theta_k; the weight 1/sqrt(1 - x_k^2) is taken as 1/sin(theta_k).
    """
    mu = np.asarray(mu, dtype=np.float64)
    M = len(mu)
    g = jackson(M) if use_jackson else np.ones(M)
    theta, x = chebyshev_points(K)
    n = np.arange(M, dtype=np.int64)[:, None]
    k = np.arange(K, dtype=np.int64)[None, :]
    m = (n * (2 * k + 1)) % (4 * K)
    cosnt = np.cos(np.pi * m / (2.0 * K))                      # (M, K)
    w = g * mu
    w[1:] *= 2.0
    f = (w[:, None] * cosnt).sum(axis=0) / (np.pi * np.sin(theta))
    return a * x + b, f / a


# --------------------------------------------------------------------------
# Green's functions from the same moments (the paper names Green's functions
# beside the DoS as targets of the expansion, Sec. I; formulas below are the
# standard Chebyshev-expansion ones of the KPM literature it cites)
# --------------------------------------------------------------------------
KERNEL_NONE, KERNEL_JACKSON, KERNEL_LORENTZ = 0, 1, 2


def lorentz(M: int, lam: float) -> np.ndarray:
    """Lorentz kernel g_n = sinh(lam (1 - n/M)) / sinh(lam), n = 0..M-1."""
    n = np.arange(M, dtype=np.float64)
    return np.sinh(lam * (1.0 - n / M)) / np.sinh(lam)


def kernel_coeffs(M: int, kernel: int, lam: float = 4.0) -> np.ndarray:
    if kernel == KERNEL_NONE:
        return np.ones(M)
    if kernel == KERNEL_JACKSON:
        return jackson(M)
    if kernel == KERNEL_LORENTZ:
        return lorentz(M, lam)
    raise ValueError(f"unknown kernel {kernel}")


def green(mu, K: int, a: float, b: float, kernel: int = KERNEL_LORENTZ, lam: float = 4.0):
    """Retarded Green's function G(omega) = <xi|(omega + i0 - H)^{-1}|xi> (per unit <xi|xi>) from the
    moments of xi, on the K Chebyshev points: with x = cos(theta), s = sin(theta),
        G~(x) = -(i/s) [g_0 mu_0 + 2 sum_{n>=1} g_n mu_n e^{-i n theta}],
    i.e. Im G~ = -(1/s) sum_n w_n cos(n theta) (= -pi f(x) of Eq. (fKPM)) and
    Re G~ = -(1/s) sum_{n>=1} w_n sin(n theta), w_n = (2 - delta_n0) g_n mu_n; then omega = a x + b and
    G(omega) = G~(x)/a.  cos and sin of n theta_k use the exact reduction m = n (2k+1) mod 4K."""
    mu = np.asarray(mu, dtype=np.float64)
    M = len(mu)
    g = kernel_coeffs(M, kernel, lam)
    theta, x = chebyshev_points(K)
    n = np.arange(M, dtype=np.int64)[:, None]
    k = np.arange(K, dtype=np.int64)[None, :]
    m = (n * (2 * k + 1)) % (4 * K)
    ang = np.pi * m / (2.0 * K)
    w = g * mu
    w[1:] *= 2.0
    fc = (w[:, None] * np.cos(ang)).sum(axis=0)
    fs = (w[:, None] * np.sin(ang)).sum(axis=0)
    s = np.sin(theta)
    return a * x + b, (-fs / s - 1j * fc / s) / a
