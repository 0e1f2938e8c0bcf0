"""paper_1105_5481_amd -- Kernel Polynomial Method hot path on MI355X (gfx950).

A thin ctypes binding over libkpm.so (C ABI in include/kpm.h).  Every step of
the computation runs in the library's HIP kernels; this module only marshals
arguments.  PyTorch supplies device memory (tensors) and streams.  If the
library is missing, every call raises KPMError: there is no fallback.
"""
from __future__ import annotations

import ctypes
import functools
import inspect
import os
from typing import List, Optional, Sequence

__all__ = [
    "KPMError", "lib", "library_path", "Hamiltonian", "gershgorin", "scale_from_bounds", "moments",
    "moments_batched", "dos", "start_vectors", "Solve", "set_launch", "get_launch", "workspace_bytes",
    "F64", "F32", "VEC_RADEMACHER", "VEC_PHASE", "VEC_UNIT",
]

F64, F32 = 0, 1
VEC_RADEMACHER, VEC_PHASE, VEC_UNIT = 0, 1, 2
KIND_SQUARE_2D, KIND_CUBIC_3D, KIND_CSR = 2, 3, 10
HOP_REAL, HOP_SPIN = 0, 1
KERNEL_NONE, KERNEL_JACKSON, KERNEL_LORENTZ = 0, 1, 2

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libkpm.so")
_lib = None


class KPMError(RuntimeError):
    pass


class HamDesc(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("hop", ctypes.c_int32), ("L", ctypes.c_int64 * 3),
                ("t", ctypes.c_double), ("onsite_dev", ctypes.c_void_p), ("spinor_dev", ctypes.c_void_p),
                ("n", ctypes.c_int64), ("nnz", ctypes.c_int64), ("row_ptr_dev", ctypes.c_void_p),
                ("col_dev", ctypes.c_void_p), ("val_re_dev", ctypes.c_void_p), ("val_im_dev", ctypes.c_void_p)]


def library_path() -> str:
    return _LIB_PATH


def lib():
    """Load libkpm.so (built in-tree by paper_1105_5481_amd/build.py)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise KPMError(f"libkpm.so not found at {_LIB_PATH}; build it with python paper_1105_5481_amd/build.py")
    # PyTorch carries its own copy of the HIP runtime (same soname, different file name on its
    # dependency list).  Loading torch first makes libkpm.so bind to that same runtime; loaded the
    # other way round, the process would hold two HIP runtimes and the second one to initialise
    # finds no device.
    _torch()
    L = ctypes.CDLL(_LIB_PATH)
    P, i32, i64, u64, f64, sz = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64,
                                 ctypes.c_double, ctypes.c_size_t)
    pdesc = ctypes.POINTER(HamDesc)
    sigs = {
        "kpm_status_string": (ctypes.c_char_p, [i32]),
        "kpm_scale_from_bounds": (i32, [f64, f64, f64, P, P]),
        "kpm_bounds_gershgorin": (i32, [pdesc, P, P]),
        "kpm_build": (i32, [pdesc, f64, f64, i32, P, P]),
        "kpm_free": (None, [P]),
        "kpm_update": (i32, [P, pdesc, f64, f64, P]),
        "kpm_ham_dim": (i64, [P]),
        "kpm_ham_get_scale": (i32, [P, P, P]),
        "kpm_workspace_bytes": (sz, [P, i32, i32, i32]),
        "kpm_moments": (i32, [P, i32, i32, i32, u64, u64, P, sz, P, P]),
        "kpm_moments_static": (i32, [P, i32, i32, i32, u64, u64, P, P]),
        "kpm_static_scratch_bytes": (sz, []),
        "kpm_solve_begin": (i32, [P, i32, i32, i32, u64, u64, P, sz, P, P]),
        "kpm_solve_advance": (i32, [P, i32, P, P]),
        "kpm_solve_finish": (i32, [P, P, P]),
        "kpm_solve_free": (None, [P]),
        "kpm_workspace_bytes_batched": (sz, [P, i32, P, P, i32]),
        "kpm_moments_batched": (i32, [P, i32, P, P, i32, P, P, P, sz, P, P]),
        "kpm_dos": (i32, [P, i32, i32, i32, f64, f64, P, P, P]),
        "kpm_start_vectors": (i32, [i32, i32, u64, u64, i64, i32, P, P]),
        "kpm_set_launch": (i32, [i32, i32]),
        "kpm_get_launch": (i32, [i32, P]),
        "kpm_selftest_fastdiv": (i32, [ctypes.c_uint32, P, i32]),
        "kpm_selftest_placement": (ctypes.c_int64, [P, P, P, i32, i32, P, P, P, ctypes.c_int64]),
        "kpm_solve_remaining": (i32, [P, P]),
        "kpm_request_bytes": (sz, [pdesc, i32, i32, i32, i32]),
        "kpm_ham_bytes": (sz, [P]),
        "kpm_batch_create": (i32, [i32, P]),
        "kpm_batch_add": (i32, [P, P]),
        "kpm_batch_remove": (i32, [P, P]),
        "kpm_batch_size": (i32, [P]),
        "kpm_batch_advance": (i32, [P, i32, P]),
        "kpm_batch_free": (None, [P]),
        "kpm_graph_capture_batched": (i32, [P, i32, P, P, i32, P, P, P, sz, P, P, P]),
        "kpm_graph_launch": (i32, [P, P]),
        "kpm_graph_free": (None, [P]),
        "kpm_lanczos_workspace_bytes": (sz, [P, i32]),
        "kpm_green": (i32, [P, i32, i32, f64, i32, f64, f64, P, P, P, P]),
        "kpm_last_hip_error": (ctypes.c_char_p, []),
        "kpm_solve_mode": (i32, [P]),
        "kpm_dense_workspace_bytes": (sz, [i64, i32, i32]),
        "kpm_dense_moments": (i32, [P, i64, f64, f64, i32, i32, i32, u64, u64, P, sz, P, P]),
        "kpm_bounds_lanczos": (i32, [P, i32, u64, f64, f64, f64, P, sz, P, P]),
    }
    for name, (res, args) in sigs.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def _check(st: int, what: str):
    if st != 0:
        msg = lib().kpm_status_string(st).decode()
        hip = lib().kpm_last_hip_error().decode()
        raise KPMError(f"{what}: {msg} (status {st}; last HIP error: {hip})")


def _torch():
    import torch
    return torch


def _stream(stream) -> ctypes.c_void_p:
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def _stream_scoped(fn):
    """Run `fn` with its `stream` argument (when given) as torch's current stream, so the tensors it
    allocates and the torch operations it issues are ordered with its library calls on that stream
    (a torch.cuda.Stream, or a raw hipStream_t handle as an int)."""
    sig = inspect.signature(fn)

    @functools.wraps(fn)
    def wrapper(*args, **kwargs):
        stream = sig.bind_partial(*args, **kwargs).arguments.get("stream")
        if stream is None:
            return fn(*args, **kwargs)
        torch = _torch()
        if not isinstance(stream, torch.cuda.Stream):
            stream = torch.cuda.ExternalStream(int(stream))
        with torch.cuda.stream(stream):
            return fn(*args, **kwargs)
    return wrapper


def _dev(x, dtype, device):
    torch = _torch()
    if x is None:
        return None
    if isinstance(x, torch.Tensor):
        return x.to(device=device, dtype=dtype).contiguous()
    import numpy as np
    return torch.from_numpy(np.ascontiguousarray(x)).to(device=device, dtype=dtype)


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _desc_for(op, device):
    """A kpm_ham_desc for a workloads.Lattice or workloads.CSR, plus the device tensors it points to."""
    torch = _torch()
    d = HamDesc()
    keep = []
    if hasattr(op, "row_ptr"):
        rp = _dev(op.row_ptr, torch.int64, device)
        cl = _dev(op.col, torch.int32, device)
        vr = _dev(op.val_re, torch.float64, device)
        vi = _dev(op.val_im, torch.float64, device) if op.val_im is not None else None
        keep += [rp, cl, vr, vi]
        d.kind = KIND_CSR
        d.n = int(op.n)
        d.nnz = int(op.row_ptr[-1])
        d.row_ptr_dev, d.col_dev, d.val_re_dev, d.val_im_dev = _ptr(rp), _ptr(cl), _ptr(vr), _ptr(vi)
    else:
        d.kind = KIND_CUBIC_3D if op.dim == 3 else KIND_SQUARE_2D
        d.hop = int(op.hop)
        d.L[0], d.L[1], d.L[2] = int(op.L[0]), int(op.L[1]), int(op.L[2]) if op.dim == 3 else 1
        d.t = float(op.t)
        on = _dev(op.onsite, torch.float64, device) if op.onsite is not None else None
        sp = _dev(op.spinor, torch.float64, device) if op.spinor is not None else None
        keep += [on, sp]
        d.onsite_dev, d.spinor_dev = _ptr(on), _ptr(sp)
    return d, keep


def scale_from_bounds(e_lo: float, e_hi: float, eps: float = 0.01):
    a, b = ctypes.c_double(), ctypes.c_double()
    _check(lib().kpm_scale_from_bounds(e_lo, e_hi, eps, ctypes.byref(a), ctypes.byref(b)), "kpm_scale_from_bounds")
    return a.value, b.value


@_stream_scoped
def gershgorin(op, device="cuda", stream=None):
    """(E_lo, E_hi) of a Lattice or CSR, computed on the device in FP64."""
    torch = _torch()
    d, keep = _desc_for(op, device)
    out = torch.empty(2, dtype=torch.float64, device=device)
    _check(lib().kpm_bounds_gershgorin(ctypes.byref(d), _ptr(out), _stream(stream)), "kpm_bounds_gershgorin")
    torch.cuda.current_stream().synchronize()
    lo, hi = out.tolist()
    return lo, hi


@_stream_scoped
def lanczos_bounds(ham: "Hamiltonian", k: int = 100, seed: int = 0, pad: float = 0.005, clamp="gershgorin",
                   stream=None) -> dict:
    """Spectral interval of H from k Lanczos steps on the FP64 operator `ham` (kpm_bounds_lanczos):
    the extreme Ritz values padded by max(residual bound, pad x their spread), mapped back through
    the operator's (a, b) and clipped to `clamp` ("gershgorin": the device Gershgorin interval of
    ham.op; None: no clipping; or an (E_lo, E_hi) pair).  Returns e_lo, e_hi, theta_min, theta_max,
    r_min, r_max (these four for H~), m (steps used) and the alpha, beta arrays."""
    torch = _torch()
    if isinstance(clamp, str) and clamp == "gershgorin":
        clamp = gershgorin(ham.op, ham.device, stream)
    lo, hi = (-float("inf"), float("inf")) if clamp is None else (float(clamp[0]), float(clamp[1]))
    nb = lib().kpm_lanczos_workspace_bytes(ham.handle, int(k))
    if nb == 0:
        raise KPMError(f"Lanczos bounds need an FP64 operator and 1 <= k <= 512 (k={k})")
    ws = _workspace(nb, ham.device)
    out = torch.empty(8 + 2 * int(k), dtype=torch.float64, device=ham.device)
    _check(lib().kpm_bounds_lanczos(ham.handle, int(k), int(seed), float(pad), lo, hi, ws.data_ptr(), nb,
                                    out.data_ptr(), _stream(stream)), "kpm_bounds_lanczos")
    o = out.cpu().numpy()
    return {"e_lo": float(o[0]), "e_hi": float(o[1]), "theta_min": float(o[2]), "theta_max": float(o[3]),
            "r_min": float(o[4]), "r_max": float(o[5]), "m": int(o[6]), "alpha": o[8:8 + k].copy(),
            "beta": o[8 + k:8 + 2 * k].copy()}


@_stream_scoped
def lanczos_scale(op, k: int = 100, eps: float = 0.01, pad: float = 0.005, seed: int = 0, device="cuda",
                  stream=None):
    """(a, b) of Eq. (tilde) from the Lanczos interval of `op` (clipped to Gershgorin), with the
    relative margin eps of scale_from_bounds."""
    h = Hamiltonian(op, 1.0, 0.0, F64, device, stream)
    try:
        r = lanczos_bounds(h, k, seed, pad, "gershgorin", stream)
    finally:
        h.free()
    return scale_from_bounds(r["e_lo"], r["e_hi"], eps)


class Hamiltonian:
    """The scaled operator H~ = (H - b)/a of Eq. (tilde), resident in device memory."""

    @_stream_scoped
    def __init__(self, op, a: float, b: float, prec: int = F64, device="cuda", stream=None):
        self.op, self.a, self.b, self.prec, self.device = op, float(a), float(b), int(prec), device
        d, keep = _desc_for(op, device)
        h = ctypes.c_void_p()
        _check(lib().kpm_build(ctypes.byref(d), self.a, self.b, self.prec, _stream(stream), ctypes.byref(h)),
               "kpm_build")
        self._h = h
        # the descriptor's arrays must live until the build kernel has run
        _torch().cuda.current_stream().synchronize()
        del keep

    @_stream_scoped
    def update(self, op, a: float, b: float, stream=None, keep_inputs: bool = False):
        """Re-prepare H~ from new inputs of the same shape in place (no allocation).  The input
        tensors are returned when keep_inputs is set (they must outlive the enqueued kernel);
        otherwise the stream is synchronised before returning."""
        d, keep = _desc_for(op, self.device)
        _check(lib().kpm_update(self.handle, ctypes.byref(d), float(a), float(b), _stream(stream)), "kpm_update")
        self.op, self.a, self.b = op, float(a), float(b)
        if keep_inputs:
            return keep
        _torch().cuda.current_stream().synchronize()
        return None

    @property
    def handle(self):
        if self._h is None:
            raise KPMError("Hamiltonian already freed")
        return self._h

    @property
    def N(self) -> int:
        return int(lib().kpm_ham_dim(self.handle))

    def scale(self):
        """(a, b) of H~ = (H - b)/a as the operator holds them (kpm_ham_get_scale)."""
        a, b = ctypes.c_double(), ctypes.c_double()
        _check(lib().kpm_ham_get_scale(self.handle, ctypes.byref(a), ctypes.byref(b)), "kpm_ham_get_scale")
        return a.value, b.value

    def workspace_bytes(self, M: int, R: int, vec: int) -> int:
        n = lib().kpm_workspace_bytes(self.handle, M, R, vec)
        if n == 0:
            raise KPMError(f"invalid solve shape M={M} R={R} vec={vec}")
        return int(n)

    def free(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().kpm_free(self._h)
        self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def workspace_bytes(ham: Hamiltonian, M: int, R: int, vec: int) -> int:
    return ham.workspace_bytes(M, R, vec)


def _workspace(nbytes: int, device, workspace=None):
    torch = _torch()
    if workspace is not None:
        if workspace.numel() * workspace.element_size() < nbytes:
            raise KPMError("workspace too small")
        return workspace
    # torch's caching allocator returns 512-byte aligned blocks
    return torch.empty(nbytes, dtype=torch.uint8, device=device)


@_stream_scoped
def moments(ham: Hamiltonian, M: int, R: int, vec: int = VEC_RADEMACHER, seed: int = 0, instance: int = 0,
            stream=None, out=None, workspace=None):
    """mu_0..mu_{M-1} (device FP64 tensor) averaged over R start vectors."""
    torch = _torch()
    nb = ham.workspace_bytes(M, R, vec)
    ws = _workspace(nb, ham.device, workspace)
    mu = out if out is not None else torch.empty(M, dtype=torch.float64, device=ham.device)
    _check(lib().kpm_moments(ham.handle, M, R, vec, seed, instance, ws.data_ptr(), nb, mu.data_ptr(),
                             _stream(stream)), "kpm_moments")
    return mu


@_stream_scoped
def moments_static(ham: Hamiltonian, M: int, R: int, vec: int = VEC_RADEMACHER, seed: int = 0, instance: int = 0,
                   stream=None, out=None):
    """mu_0..mu_{M-1} like `moments`, run in the library's static device scratch (kpm_moments_static:
    no device allocation by the library; pass `out` to avoid torch's as well)."""
    torch = _torch()
    mu = out if out is not None else torch.empty(M, dtype=torch.float64, device=ham.device)
    _check(lib().kpm_moments_static(ham.handle, M, R, vec, seed, instance, mu.data_ptr(), _stream(stream)),
           "kpm_moments_static")
    return mu


@_stream_scoped
def moments_batched(hams: Sequence[Hamiltonian], M, R, vec: int = VEC_RADEMACHER, seeds=None, instances=None,
                    stream=None, outs=None, workspace=None) -> List:
    torch = _torch()
    n = len(hams)
    Ms = [int(M)] * n if isinstance(M, int) else [int(x) for x in M]
    Rs = [int(R)] * n if isinstance(R, int) else [int(x) for x in R]
    seeds = [0] * n if seeds is None else list(seeds)
    instances = list(range(n)) if instances is None else list(instances)
    harr = (ctypes.c_void_p * n)(*[h.handle.value for h in hams])
    marr = (ctypes.c_int32 * n)(*Ms)
    rarr = (ctypes.c_int32 * n)(*Rs)
    sarr = (ctypes.c_uint64 * n)(*seeds)
    iarr = (ctypes.c_uint64 * n)(*instances)
    nb = lib().kpm_workspace_bytes_batched(harr, n, marr, rarr, vec)
    if nb == 0:
        raise KPMError("invalid batch")
    ws = _workspace(nb, hams[0].device, workspace)
    mus = outs if outs is not None else [torch.empty(m, dtype=torch.float64, device=hams[0].device) for m in Ms]
    parr = (ctypes.c_void_p * n)(*[m.data_ptr() for m in mus])
    _check(lib().kpm_moments_batched(harr, n, marr, rarr, vec, sarr, iarr, ws.data_ptr(), nb, parr,
                                     _stream(stream)), "kpm_moments_batched")
    return mus


class BatchedGraph:
    """A batched solve captured once into a hipGraph and replayed (kpm_graph_capture_batched).
    `stream` must be a non-default torch.cuda.Stream; outputs land in self.mus on every replay."""

    def __init__(self, hams: Sequence[Hamiltonian], M, R, vec: int, seeds, instances, stream):
        torch = _torch()
        n = len(hams)
        self.hams = list(hams)
        self.Ms = [int(M)] * n if isinstance(M, int) else [int(x) for x in M]
        self.Rs = [int(R)] * n if isinstance(R, int) else [int(x) for x in R]
        self._harr = (ctypes.c_void_p * n)(*[h.handle.value for h in hams])
        self._marr = (ctypes.c_int32 * n)(*self.Ms)
        self._rarr = (ctypes.c_int32 * n)(*self.Rs)
        self._sarr = (ctypes.c_uint64 * n)(*list(seeds))
        self._iarr = (ctypes.c_uint64 * n)(*list(instances))
        nb = lib().kpm_workspace_bytes_batched(self._harr, n, self._marr, self._rarr, vec)
        if nb == 0:
            raise KPMError("invalid batch")
        self.ws = torch.empty(nb, dtype=torch.uint8, device=hams[0].device)
        self.mus = [torch.empty(m, dtype=torch.float64, device=hams[0].device) for m in self.Ms]
        self._parr = (ctypes.c_void_p * n)(*[m.data_ptr() for m in self.mus])
        self.stream = stream
        g = ctypes.c_void_p()
        _check(lib().kpm_graph_capture_batched(self._harr, n, self._marr, self._rarr, vec, self._sarr, self._iarr,
                                               self.ws.data_ptr(), nb, self._parr, _stream(stream), ctypes.byref(g)),
               "kpm_graph_capture_batched")
        self._g = g

    def launch(self):
        _check(lib().kpm_graph_launch(self._g, _stream(self.stream)), "kpm_graph_launch")
        return self.mus

    def free(self):
        if getattr(self, "_g", None) is not None and self._g.value:
            lib().kpm_graph_free(self._g)
        self._g = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Solve:
    """A chunked solve: begin -> advance(k) ... -> finish; the vector state stays in `workspace`."""

    @_stream_scoped
    def __init__(self, ham: Hamiltonian, M: int, R: int, vec: int = VEC_RADEMACHER, seed: int = 0,
                 instance: int = 0, stream=None, workspace=None):
        self.ham, self.M = ham, M
        self.nbytes = ham.workspace_bytes(M, R, vec)
        self.ws = _workspace(self.nbytes, ham.device, workspace)
        s = ctypes.c_void_p()
        _check(lib().kpm_solve_begin(ham.handle, M, R, vec, seed, instance, self.ws.data_ptr(), self.nbytes,
                                     _stream(stream), ctypes.byref(s)), "kpm_solve_begin")
        self._s = s

    @property
    def remaining(self) -> int:
        rem = ctypes.c_int32()
        _check(lib().kpm_solve_remaining(self._s, ctypes.byref(rem)), "kpm_solve_remaining")
        return rem.value

    @_stream_scoped
    def advance(self, steps: int, stream=None) -> int:
        rem = ctypes.c_int32()
        _check(lib().kpm_solve_advance(self._s, steps, _stream(stream), ctypes.byref(rem)), "kpm_solve_advance")
        return rem.value

    @_stream_scoped
    def finish(self, out=None, stream=None):
        torch = _torch()
        mu = out if out is not None else torch.empty(self.M, dtype=torch.float64, device=self.ham.device)
        _check(lib().kpm_solve_finish(self._s, mu.data_ptr(), _stream(stream)), "kpm_solve_finish")
        return mu

    def close(self):
        if getattr(self, "_s", None) is not None and self._s.value:
            lib().kpm_solve_free(self._s)
        self._s = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """A dynamic batch of begun solves advanced together (continuous batching)."""

    def __init__(self, capacity: int = 256):
        b = ctypes.c_void_p()
        _check(lib().kpm_batch_create(capacity, ctypes.byref(b)), "kpm_batch_create")
        self._b = b
        self.members = []

    def add(self, solve: "Solve"):
        _check(lib().kpm_batch_add(self._b, solve._s), "kpm_batch_add")
        self.members.append(solve)

    def remove(self, solve: "Solve"):
        _check(lib().kpm_batch_remove(self._b, solve._s), "kpm_batch_remove")
        self.members.remove(solve)

    @_stream_scoped
    def advance(self, steps: int, stream=None):
        _check(lib().kpm_batch_advance(self._b, steps, _stream(stream)), "kpm_batch_advance")

    def __len__(self):
        return int(lib().kpm_batch_size(self._b))

    def free(self):
        if getattr(self, "_b", None) is not None and self._b.value:
            lib().kpm_batch_free(self._b)
        self._b = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def request_bytes(op, prec: int, M: int, R: int, vec: int) -> int:
    """Device bytes an operator plus one solve of (M, R, vec) would occupy (host-only query)."""
    d = HamDesc()
    if hasattr(op, "row_ptr"):
        d.kind, d.n, d.nnz = KIND_CSR, int(op.n), int(op.row_ptr[-1])
        d.row_ptr_dev = 1                      # only checked for presence
        d.col_dev = d.val_re_dev = 1 if d.nnz else None
        d.val_im_dev = 1 if op.val_im is not None else None
    else:
        d.kind = KIND_CUBIC_3D if op.dim == 3 else KIND_SQUARE_2D
        d.hop = int(op.hop)
        d.L[0], d.L[1], d.L[2] = int(op.L[0]), int(op.L[1]), int(op.L[2]) if op.dim == 3 else 1
        d.t = float(op.t)
        d.spinor_dev = 1 if op.spinor is not None else None
    n = lib().kpm_request_bytes(ctypes.byref(d), prec, M, R, vec)
    if n == 0:
        raise KPMError("invalid request shape")
    return int(n)


@_stream_scoped
def dos(mu, K: int, a: float, b: float, jackson: bool = True, stream=None):
    """(omega, rho) device tensors of Eq. (fKPM) on K Chebyshev points."""
    torch = _torch()
    M = mu.numel()
    om = torch.empty(K, dtype=torch.float64, device=mu.device)
    rho = torch.empty(K, dtype=torch.float64, device=mu.device)
    _check(lib().kpm_dos(mu.data_ptr(), M, 1 if jackson else 0, K, float(a), float(b), om.data_ptr(),
                         rho.data_ptr(), _stream(stream)), "kpm_dos")
    return om, rho


@_stream_scoped
def dense_moments(H, a: float, b: float, M: int, R: int, vec: int = VEC_RADEMACHER, seed: int = 0, instance: int = 0,
                  stream=None, out=None, workspace=None):
    """Moments of a dense real symmetric H (a D x D float64 device tensor, row-major) on the matrix
    cores (kpm_dense_moments); returns a device tensor of M doubles."""
    torch = _torch()
    if H.dtype != torch.float64 or H.dim() != 2 or H.shape[0] != H.shape[1] or not H.is_contiguous():
        raise KPMError("dense_moments needs a contiguous square float64 tensor")
    D = H.shape[0]
    nb = lib().kpm_dense_workspace_bytes(D, int(M), int(R))
    if nb == 0:
        raise KPMError(f"invalid dense solve shape D={D} M={M} R={R}")
    ws = _workspace(nb, H.device, workspace)
    mu = out if out is not None else torch.empty(int(M), dtype=torch.float64, device=H.device)
    _check(lib().kpm_dense_moments(H.data_ptr(), D, float(a), float(b), int(M), int(R), int(vec), int(seed),
                                   int(instance), ws.data_ptr(), nb, mu.data_ptr(), _stream(stream)),
           "kpm_dense_moments")
    return mu


@_stream_scoped
def green(mu, K: int, a: float, b: float, kernel: int = KERNEL_LORENTZ, lam: float = 4.0, stream=None):
    """(omega, G) device tensors (G complex128) of the Green's function <xi|(omega + i0 - H)^{-1}|xi>
    from the moments of xi (kpm_green) on K Chebyshev points."""
    torch = _torch()
    M = mu.numel()
    om = torch.empty(K, dtype=torch.float64, device=mu.device)
    gre = torch.empty(K, dtype=torch.float64, device=mu.device)
    gim = torch.empty(K, dtype=torch.float64, device=mu.device)
    _check(lib().kpm_green(mu.data_ptr(), M, int(kernel), float(lam), K, float(a), float(b), om.data_ptr(),
                           gre.data_ptr(), gim.data_ptr(), _stream(stream)), "kpm_green")
    return om, torch.complex(gre, gim)


@_stream_scoped
def site_moments(ham: "Hamiltonian", sites, M: int, stream=None) -> List:
    """Moments <i|T_n(H~)|i> of the local DoS at each site i (unit start vector e_i): one batched
    solve with R = 1 per site (KPM_VEC_UNIT with instance = i)."""
    sites = [int(i) for i in sites]
    if not sites:
        return []
    N = ham.N
    if min(sites) < 0 or max(sites) >= N:
        raise KPMError(f"site index out of range [0, {N})")
    return moments_batched([ham] * len(sites), M, 1, VEC_UNIT, [0] * len(sites), sites, stream=stream)


@_stream_scoped
def ldos(ham: "Hamiltonian", sites, M: int, K: Optional[int] = None, jackson: bool = True, stream=None):
    """Local DoS rho_i(omega) at each site: (omega [K], rho [len(sites), K]) device tensors."""
    torch = _torch()
    K = K or 2 * M
    mus = site_moments(ham, sites, M, stream)
    rows = []
    om = None
    for mu in mus:
        om, rho = dos(mu, K, ham.a, ham.b, jackson, stream)
        rows.append(rho)
    return om, torch.stack(rows) if rows else None


@_stream_scoped
def site_green(ham: "Hamiltonian", sites, M: int, K: Optional[int] = None, kernel: int = KERNEL_LORENTZ,
               lam: float = 4.0, stream=None):
    """Site-diagonal Green's functions G_ii(omega + i0): (omega [K], G [len(sites), K] complex)."""
    torch = _torch()
    K = K or 2 * M
    mus = site_moments(ham, sites, M, stream)
    rows = []
    om = None
    for mu in mus:
        om, G = green(mu, K, ham.a, ham.b, kernel, lam, stream)
        rows.append(G)
    return om, torch.stack(rows) if rows else None


@_stream_scoped
def start_vectors(vec: int, complex_layout: bool, seed: int, instance: int, N: int, R: int, device="cuda",
                  stream=None):
    torch = _torch()
    cplx = complex_layout or vec == VEC_PHASE
    out = torch.empty((N, R, 2) if cplx else (N, R), dtype=torch.float64, device=device)
    _check(lib().kpm_start_vectors(vec, 1 if cplx else 0, seed, instance, N, R, out.data_ptr(), _stream(stream)),
           "kpm_start_vectors")
    return out


LAUNCH_ELEMS_PER_THREAD, LAUNCH_MAX_BLOCKS, LAUNCH_MARCH, LAUNCH_MARCH_ITEMS, LAUNCH_XCD_SPLIT, LAUNCH_ALTERNATE, \
    LAUNCH_SMALL, LAUNCH_STREAMING = range(8)
_LAUNCH_KEYS = {"elems_per_thread": 0, "max_blocks": 1, "march": 2, "march_items": 3, "xcd_split": 4, "alternate": 5,
                "small": 6, "streaming": 7, "wave_mib": 8, "tblock": 9, "tb3": 10, "tb_group": 11}


def set_launch(**kw):
    """Launch-shape tuning, e.g. set_launch(max_blocks=4096, march=1, march_items=2048)."""
    for k, v in kw.items():
        if v is None:
            continue
        _check(lib().kpm_set_launch(_LAUNCH_KEYS[k], int(v)), f"kpm_set_launch({k}={v})")


def get_launch() -> dict:
    out = {}
    for k, key in _LAUNCH_KEYS.items():
        v = ctypes.c_int32()
        _check(lib().kpm_get_launch(key, ctypes.byref(v)), "kpm_get_launch")
        out[k] = v.value
    return out


class launch_settings:
    """Context manager applying set_launch(**kw) and restoring the previous settings."""

    def __init__(self, **kw):
        self.kw = kw

    def __enter__(self):
        self.old = get_launch()
        set_launch(**self.kw)
        return self

    def __exit__(self, *exc):
        set_launch(**self.old)
        return False
