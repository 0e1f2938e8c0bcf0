"""Full-size parity: the workloads the benchmark runs, against stored oracle moments.

tests/golden/*_oracle.txt are written by tests/golden/make_golden.py, which calls only the CPU
oracle.  FP64 must match to REL64 (relative, floor FLOOR64); FP32/complex64 to ABS32 per moment.
The FP32 DoS error is reported as an L1 distance (Gauss-Chebyshev quadrature over omega), which
is bounded by 2 sum_n g_n |d mu_n| (the kernel-damped expansion of the moment error).
"""
import os

import numpy as np
import pytest

import oracle
import paper_1105_5481_amd as kpm
from paper_1105_5481_amd import workloads as wl
from tests import gpu_util as gu
from tests.golden.make_golden import load

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def golden(name):
    path = os.path.join(GOLDEN, name)
    if not os.path.exists(path):
        pytest.skip(f"{name} not generated (python tests/golden/make_golden.py)")
    hdr, mu = load(path)
    return hdr, np.array(mu), float.fromhex(hdr["a"]), float.fromhex(hdr["b"])


def dos_l1(mu_a, mu_b, K, a, b):
    import torch
    _, ra = kpm.dos(torch.from_numpy(np.ascontiguousarray(mu_a)).cuda(), K, a, b)
    _, rb = kpm.dos(torch.from_numpy(np.ascontiguousarray(mu_b)).cuda(), K, a, b)
    theta = np.pi * (np.arange(K) + 0.5) / K
    w = a * np.pi / K * np.sin(theta)                       # d omega = a dx, dx = (pi/K) sin(theta_k)
    l1 = float(np.sum(np.abs(ra.cpu().numpy() - rb.cpu().numpy()) * w))
    g = oracle.jackson(len(mu_a))
    bound = float(g[0] * abs(mu_a[0] - mu_b[0]) + 2 * np.sum(g[1:] * np.abs(mu_a[1:] - mu_b[1:])))
    return l1, bound


def test_config2_full():
    hdr, ref, a, b = golden("config2_oracle.txt")
    cfg = wl.config2()
    lat = cfg["lattice"]
    lo, hi = kpm.gershgorin(lat)
    assert abs(kpm.scale_from_bounds(lo, hi, 0.01)[0] - a) <= 4e-16 * a
    M, R = int(hdr["M"]), int(hdr["R"])
    g64 = gu.gpu_moments(lat, a, b, kpm.F64, M, R, cfg["vec"], cfg["seed"], 0)
    gu.assert_fp64(g64, ref, "config2 c128")
    g32 = gu.gpu_moments(lat, a, b, kpm.F32, M, R, cfg["vec"], cfg["seed"], 0)
    gu.assert_fp32(g32, ref, "config2 c64")
    l1, bound = dos_l1(g32, ref, 2 * M, a, b)
    print(f"  config2 c64 DoS L1 error {l1:.3e} (bound {bound:.3e})")
    assert l1 <= bound * (1 + 1e-9) + 1e-15


def test_config4_full():
    """The full M=4096 FP32 solve (temporally blocked passes) against the oracle on every stored
    moment, its DoS L1 error against the bound, and the FP64 path (three-step passes) on the same
    moments at REL64."""
    hdr, ref, a, b = golden("config4_oracle.txt")
    cfg = wl.config4()
    lat = cfg["lattice"]
    Mref = len(ref)
    print(f"  config4 golden: {Mref} of {cfg['M']} moments", flush=True)
    g32 = gu.gpu_moments(lat, a, b, kpm.F32, cfg["M"], cfg["R"], cfg["vec"], cfg["seed"], 0)
    gu.assert_fp32(g32[:Mref], ref, f"config4 f32 (first {Mref} of M=4096)")
    assert np.all(np.isfinite(g32)) and np.abs(g32).max() <= 1.0 + 1e-6
    if Mref == cfg["M"]:
        l1, bound = dos_l1(g32, ref, 2 * cfg["M"], a, b)
        print(f"  config4 f32 DoS L1 error {l1:.3e} (bound {bound:.3e})", flush=True)
        assert l1 <= bound * (1 + 1e-9) + 1e-15
    g64 = gu.gpu_moments(lat, a, b, kpm.F64, Mref, cfg["R"], cfg["vec"], cfg["seed"], 0)
    gu.assert_fp64(g64, ref, f"config4 f64 M={Mref}")


def test_config3_batch():
    """All 256 cubes in one batched c64 solve; every instance with stored oracle moments (the first
    four, every L=48 cube and a spread of other sizes) against the oracle, each equal (bitwise) to
    the same instance solved alone, and its c128 path against the oracle at REL64."""
    from tests.golden.make_golden import CONFIG3_EXTRA
    cfg = wl.config3()
    M, R, vec, seed = cfg["M"], cfg["R"], cfg["vec"], cfg["seed"]
    checked = [h for h in list(range(4)) + list(CONFIG3_EXTRA)
               if os.path.exists(os.path.join(GOLDEN, f"config3_h{h}_oracle.txt"))]
    assert len(checked) >= 4
    refs = {h: golden(f"config3_h{h}_oracle.txt") for h in checked}
    hs = []
    for h, lat in enumerate(cfg["lattices"]):
        if h in refs:
            a, b = refs[h][2], refs[h][3]
        else:
            lo, hi = kpm.gershgorin(lat)
            a, b = kpm.scale_from_bounds(lo, hi, 0.01)
        hs.append(kpm.Hamiltonian(lat, a, b, kpm.F32))
    mus = [m.cpu().numpy() for m in kpm.moments_batched(hs, M, R, vec, [seed] * len(hs), list(range(len(hs))))]
    for h in checked:
        L = cfg["lattices"][h].L[0]
        gu.assert_fp32(mus[h], refs[h][1], f"config3 batched c64 instance {h} (L={L})")
        solo = kpm.moments(hs[h], M, R, vec, seed, h).cpu().numpy()
        assert np.array_equal(solo, mus[h])
        g64 = gu.gpu_moments(cfg["lattices"][h], refs[h][2], refs[h][3], kpm.F64, M, R, vec, seed, h)
        gu.assert_fp64(g64, refs[h][1], f"config3 c128 instance {h} (L={L})")
    assert any(cfg["lattices"][h].L[0] == 48 for h in checked)
    assert all(np.all(np.isfinite(m)) and abs(m[0] - 1.0) < 1e-6 for m in mus)
    for h in hs:
        h.free()
