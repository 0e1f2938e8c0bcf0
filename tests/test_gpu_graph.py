"""A batched solve captured into a hipGraph: every replay equals the eager result bit for bit,
also after the operators are re-prepared in place between replays (Monte-Carlo style)."""
import numpy as np
import pytest

import oracle
import paper_1105_5481_amd as kpm
from paper_1105_5481_amd import workloads as wl
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu


def _batch():
    ops = [wl.spin_cubic_lattice(L, seed=60 + L) for L in (6, 12, 17)]
    ops.append(wl.square_lattice(70, W=1.0, seed=64))
    ops.append(wl.lattice_to_csr(wl.square_lattice(30, W=1.0, seed=65)))
    return ops


@pytest.mark.parametrize("prec", [kpm.F64, kpm.F32])
def test_graph_replays_equal_eager(prec):
    import torch
    ops = _batch()
    hs = []
    for op in ops:
        lo, hi = gu.oracle_bounds(op)
        a, b = oracle.scale_from_bounds(lo, hi, 0.01)
        hs.append(kpm.Hamiltonian(op, a, b, prec))
    Ms, Rs = [64, 96, 128, 80, 50], [3, 4, 5, 6, 2]
    seeds, insts = [1, 2, 3, 4, 5], [0, 1, 2, 3, 4]
    eager = [m.cpu().numpy() for m in kpm.moments_batched(hs, Ms, Rs, wl.VEC_PHASE, seeds, insts)]
    side = torch.cuda.Stream()
    g = kpm.BatchedGraph(hs, Ms, Rs, wl.VEC_PHASE, seeds, insts, side)
    for rep in range(3):
        mus = g.launch()
        side.synchronize()
        got = [m.cpu().numpy() for m in mus]
        for k in range(len(hs)):
            assert np.array_equal(got[k], eager[k]), (rep, k)
        # eager work of the program between replays
        x = torch.randn(1 << 20, device="cuda")
        torch.cuda.synchronize()
        assert torch.isfinite(x.sum())
    # Monte-Carlo step: re-draw a few spins of instance 1, re-prepare in place, replay
    op1 = ops[1]
    th, ph = op1.theta.copy(), op1.phi.copy()
    th[:5] = np.pi - th[:5]
    ph[:5] = ph[:5] + 1.0
    new = wl.spin_cubic_lattice(op1.L[0], theta=th, phi=ph)
    hs[1].update(new, hs[1].a, hs[1].b)
    mus = g.launch()
    side.synchronize()
    solo = kpm.moments(hs[1], Ms[1], Rs[1], wl.VEC_PHASE, seeds[1], insts[1]).cpu().numpy()
    assert np.array_equal(mus[1].cpu().numpy(), solo)
    assert not np.array_equal(solo, eager[1])
    if prec == kpm.F64:
        ref = gu.oracle_moments(new, hs[1].a, hs[1].b, Ms[1], Rs[1], wl.VEC_PHASE, seeds[1], insts[1])
        gu.assert_fp64(solo, ref, "updated operator")
    g.free()
    for h in hs:
        h.free()
