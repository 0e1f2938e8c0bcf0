"""FP32 recursion at the largest moment count a request may ask for (M = 8192) on small lattices
(N = 4096), against the FP64 oracle.

Rounding errors of the FP32 vectors accumulate over the 4096 recursion steps of Eq. (rn), and on a
small lattice the stochastic trace averages over few sites, so this corner bounds the FP32 error of
every moment of Eq. (munr) from above for the request mix.  Each case runs the path the library
picks for it (temporally blocked 2D passes, or one-step march kernels) and also checks the FP64 path
on the same operator.  The scale is the Gershgorin interval with margin 0.01, a and b taken as they
are (no rounding to FP32 values).
"""
import numpy as np
import pytest

import oracle
import paper_1105_5481_amd as kpm
from paper_1105_5481_amd import workloads as wl
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu

M_LONG = 8192
R_LONG = 8


def _spin2d(Lx, Ly, seed):
    th, ph = wl.spins_uniform(Lx * Ly, seed)
    return wl.Lattice(dim=2, L=(Lx, Ly, 1), t=1.0, hop=wl.HOP_SPIN, spinor=wl.spinor_of(th, ph), theta=th, phi=ph)


def _cases():
    return [
        # (name, lattice, vector kind, solve mode expected for FP32: 3 blocked 2D, 4 blocked 3D, 1 march)
        ("square_256x16_anderson_pm1", wl.Lattice(dim=2, L=(256, 16, 1), t=1.0,
                                                   onsite=wl.anderson_onsite(4096, 2.0, 41)), wl.VEC_RADEMACHER, 3),
        ("spin2d_128x32_phase", _spin2d(128, 32, 42), wl.VEC_PHASE, 3),
        ("spin2d_64x64_phase", _spin2d(64, 64, 43), wl.VEC_PHASE, 1),
        ("spin3d_16_phase", wl.spin_cubic_lattice(16, seed=44), wl.VEC_PHASE, 1),
        ("cubic_16_anderson_pm1", wl.cubic_lattice(16, t=1.0, W=1.0, seed=45), wl.VEC_RADEMACHER, 4),
    ]


@pytest.fixture(scope="module", autouse=True)
def _setup():
    import torch
    assert torch.cuda.is_available()
    kpm.lib()
    oracle.build()
    yield


def _mode(h, M, R, vec):
    """The solve mode the library chooses for this operator and shape."""
    import ctypes
    import torch
    L = kpm.lib()
    nb = h.workspace_bytes(M, R, vec)
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    s = ctypes.c_void_p()
    sp = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    kpm._check(L.kpm_solve_begin(h.handle, M, R, vec, 1, 0, ws.data_ptr(), nb, sp, ctypes.byref(s)), "begin")
    m = L.kpm_solve_mode(s)
    L.kpm_solve_free(s)
    torch.cuda.synchronize()
    return m


@pytest.mark.parametrize("case", _cases(), ids=lambda c: c[0])
def test_fp32_long_recursion(case):
    name, lat, vec, mode = case
    print(f"\n  case {name} N={lat.N} M={M_LONG} R={R_LONG}", flush=True)
    lo, hi = gu.oracle_bounds(lat)
    a, b = oracle.scale_from_bounds(lo, hi, 0.01)
    seed = 4100
    ref = gu.oracle_moments(lat, a, b, M_LONG, R_LONG, vec, seed)
    h = kpm.Hamiltonian(lat, a, b, kpm.F32)
    assert _mode(h, M_LONG, R_LONG, vec) == mode
    g32 = kpm.moments(h, M_LONG, R_LONG, vec, seed).cpu().numpy()
    h.free()
    d = np.abs(g32 - ref)
    worst = int(np.argmax(d))
    print(f"  {name}: FP32 max|d mu| = {d.max():.3e} at n = {worst}; mean over n >= 4096: "
          f"{d[4096:].mean():.3e}", flush=True)
    gu.assert_fp32(g32, ref, name + " f32 M=8192")
    g64 = gu.gpu_moments(lat, a, b, kpm.F64, M_LONG, R_LONG, vec, seed)
    gu.assert_fp64(g64, ref, name + " f64 M=8192")
