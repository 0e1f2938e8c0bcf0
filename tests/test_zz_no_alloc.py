"""kpm_moments_static (the entry point that allocates nothing, for callers that cannot allocate)
through the C ABI, against kpm_moments with a caller workspace on the same inputs.

Two calls in a row share the library's static scratch: the first a temporally blocked 2D solve
(four vector buffers), the second a smaller 3D spin solve, so the second runs over what the first
left behind.  Each must equal kpm_moments bitwise (same kernels, same work items); one case is
also checked against the oracle.  A solve whose workspace exceeds the scratch is refused before
anything is enqueued.
"""
import ctypes

import numpy as np
import pytest

import oracle
import paper_1105_5481_amd as kpm
from paper_1105_5481_amd import workloads as wl
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu


def _static_call(L, h, M, R, vec, seed, instance, mu, stream):
    return L.kpm_moments_static(h.handle, M, R, vec, seed, instance, ctypes.c_void_p(mu.data_ptr()),
                                ctypes.c_void_p(stream.cuda_stream))


def _workspace_call(L, h, M, R, vec, seed, instance, mu, stream):
    import torch
    nb = L.kpm_workspace_bytes(h.handle, M, R, vec)
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    st = L.kpm_moments(h.handle, M, R, vec, seed, instance, ctypes.c_void_p(ws.data_ptr()), nb,
                       ctypes.c_void_p(mu.data_ptr()), ctypes.c_void_p(stream.cuda_stream))
    stream.synchronize()
    return st


def test_static_scratch_matches_workspace_path():
    import torch
    assert torch.cuda.is_available()
    L = kpm.lib()
    cap = int(L.kpm_static_scratch_bytes())
    assert cap == 64 << 20
    stream = torch.cuda.current_stream()
    big = wl.Lattice(dim=2, L=(256, 24, 1), t=1.0, onsite=wl.anderson_onsite(256 * 24, 2.0, 51))
    small = wl.spin_cubic_lattice(9, seed=52)
    cases = [  # (name, lattice, precision, M, R, vector kind, seed, instance): largest first
        ("square_256x24_f32_blocked", big, kpm.F32, 200, 16, wl.VEC_RADEMACHER, 61, 0),
        ("spin_cube_9_c128", small, kpm.F64, 90, 5, wl.VEC_PHASE, 62, 3),
        ("spin_cube_9_c64", small, kpm.F32, 64, 3, wl.VEC_PHASE, 63, 1),
    ]
    for name, lat, prec, M, R, vec, seed, inst in cases:
        print(f"  case {name}: N={lat.N} M={M} R={R}", flush=True)
        lo, hi = gu.oracle_bounds(lat)
        a, b = oracle.scale_from_bounds(lo, hi, 0.01)
        h = kpm.Hamiltonian(lat, a, b, prec)
        need = int(L.kpm_workspace_bytes(h.handle, M, R, vec))
        assert 0 < need <= cap
        mu_s = torch.full((M,), 7.0, dtype=torch.float64, device="cuda")
        mu_w = torch.full((M,), -7.0, dtype=torch.float64, device="cuda")
        assert _static_call(L, h, M, R, vec, seed, inst, mu_s, stream) == 0
        stream.synchronize()
        assert _workspace_call(L, h, M, R, vec, seed, inst, mu_w, stream) == 0
        a_s, a_w = mu_s.cpu().numpy(), mu_w.cpu().numpy()
        assert np.array_equal(a_s, a_w), (name, float(np.abs(a_s - a_w).max()))
        if name.endswith("c128"):
            ref = gu.oracle_moments(lat, a, b, M, R, vec, seed, inst)
            gu.assert_fp64(a_s, ref, name + " static scratch")
        h.free()


def test_static_scratch_refuses_oversized_solve():
    import torch
    L = kpm.lib()
    stream = torch.cuda.current_stream()
    lat = wl.square_lattice(512, W=1.0, seed=53)
    h = kpm.Hamiltonian(lat, 4.6, 0.0, kpm.F32)
    M, R = 64, 64
    assert L.kpm_workspace_bytes(h.handle, M, R, wl.VEC_RADEMACHER) > L.kpm_static_scratch_bytes()
    mu = torch.full((M,), 3.0, dtype=torch.float64, device="cuda")
    assert _static_call(L, h, M, R, wl.VEC_RADEMACHER, 1, 0, mu, stream) == 6   # KPM_ERR_WORKSPACE
    stream.synchronize()
    assert torch.all(mu == 3.0)
    assert L.kpm_moments_static(None, M, R, 0, 1, 0, ctypes.c_void_p(mu.data_ptr()), None) == 1
    h.free()
