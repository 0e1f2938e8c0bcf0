"""Temporal blocking (two, or three, recursion steps per pass) on 2D real lattices: the vectors
are bitwise those of the one-step recursion, so FP64 moments match the oracle to the usual bar and
both precisions match the one-step path; step counts and chunk sizes that are not multiples of the
pass depth exercise the pair and single-step passes between deeper ones."""
import numpy as np
import pytest

import oracle
import paper_1105_5481_amd as kpm
from paper_1105_5481_amd import workloads as wl
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu

CASES = [  # (Lx, Ly, W, R, prec, M): C = 4, 1, 16, 16 chunks per site -> windows of 128, 512, 32, 32 sites
    (300, 40, 1.0, 8, kpm.F64, 64),
    (1024, 9, 0.0, 2, kpm.F64, 33),
    (130, 70, 2.0, 64, kpm.F32, 101),
    (64, 64, 1.0, 64, kpm.F32, 40),
    (200, 30, 1.0, 8, kpm.F64, 1),     # start vectors only
    (200, 30, 1.0, 8, kpm.F64, 2),     # one single step
    (200, 30, 1.0, 8, kpm.F64, 5),     # a pair and a single step
    (200, 30, 1.0, 8, kpm.F64, 7),     # one triple (three-step passes)
    (200, 30, 1.0, 8, kpm.F32, 9),     # a triple and a single step
]
DEPTHS = [1, 3, 4, 5, 6]   # KPM_LAUNCH_TBLOCK: steps per pass (1 means two)


def _lat(Lx, Ly, W, seed):
    onsite = wl.anderson_onsite(Lx * Ly, W, seed) if W > 0 else None
    return wl.Lattice(dim=2, L=(Lx, Ly, 1), t=1.0, onsite=onsite)


@pytest.mark.parametrize("tb", DEPTHS)
@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0]}x{c[1]}-R{c[3]}-{'f64' if c[4] == 0 else 'f32'}-M{c[5]}")
def test_tblock_matches_oracle_and_one_step(case, tb):
    Lx, Ly, W, R, prec, M = case
    op = _lat(Lx, Ly, W, Lx + Ly)
    lo, hi = gu.oracle_bounds(op)
    a, b = oracle.scale_from_bounds(lo, hi, 0.01)
    with kpm.launch_settings(small=0, tblock=tb):
        tb = gu.gpu_moments(op, a, b, prec, M, R, wl.VEC_RADEMACHER, seed=5)
    with kpm.launch_settings(small=0, tblock=0):
        one = gu.gpu_moments(op, a, b, prec, M, R, wl.VEC_RADEMACHER, seed=5)
    ref = gu.oracle_moments(op, a, b, M, R, wl.VEC_RADEMACHER, 5)
    print(f"  tblock vs one-step {np.abs(tb - one).max():.2e}, vs oracle {np.abs(tb - ref).max():.2e}")
    if prec == kpm.F64:
        gu.assert_fp64(tb, ref, "temporal blocking")
        assert np.abs(tb - one).max() <= 1e-15
    else:
        gu.assert_fp32(tb, ref, "temporal blocking")
        assert np.abs(tb - one).max() <= 1e-12


@pytest.mark.parametrize("tb", DEPTHS)
@pytest.mark.parametrize("chunks", [[1, 1, 3, 2, 5, 100], [3, 3, 3, 100], [2, 100], [4, 1, 7, 100]])
def test_tblock_chunked_advance(chunks, tb):
    """Passes of every depth between the others (chunk sizes not multiples of the depth) keep the
    buffers and dots consistent."""
    import torch
    op = _lat(300, 40, 1.0, 9)
    lo, hi = gu.oracle_bounds(op)
    a, b = oracle.scale_from_bounds(lo, hi, 0.01)
    M, R = 41, 8
    with kpm.launch_settings(small=0, tblock=tb):
        h = kpm.Hamiltonian(op, a, b, kpm.F64)
        s = kpm.Solve(h, M, R, wl.VEC_RADEMACHER, 3, 0)
        for c in chunks:
            if s.remaining == 0:
                break
            s.advance(c)
        mu = s.finish().cpu().numpy()
        s.close()
        h.free()
    ref = gu.oracle_moments(op, a, b, M, R, wl.VEC_RADEMACHER, 3)
    gu.assert_fp64(mu, ref, f"chunks {chunks}")


@pytest.mark.parametrize("tb", DEPTHS)
def test_tblock_in_a_dynamic_batch(tb):
    """A temporally blocked solve advanced inside a dynamic batch beside a one-step solve."""
    op1 = _lat(300, 40, 1.0, 11)
    op2 = wl.spin_cubic_lattice(14, seed=12)
    outs = []
    with kpm.launch_settings(small=0, tblock=tb):
        hs, ss = [], []
        for op in (op1, op2):
            lo, hi = gu.oracle_bounds(op)
            a, b = oracle.scale_from_bounds(lo, hi, 0.01)
            h = kpm.Hamiltonian(op, a, b, kpm.F64)
            hs.append(h)
            ss.append(kpm.Solve(h, 50, 4, wl.VEC_PHASE, 7, 1))
        batch = kpm.Batch(capacity=4)
        for s in ss:
            batch.add(s)
        while any(s.remaining > 0 for s in ss):
            batch.advance(7)
        for s in ss:
            batch.remove(s)
            outs.append(s.finish().cpu().numpy())
            s.close()
        batch.free()
    for op, h, mu in zip((op1, op2), hs, outs):
        ref = gu.oracle_moments(op, h.a, h.b, 50, 4, wl.VEC_PHASE, 7, 1)
        gu.assert_fp64(mu, ref, "batched")
        h.free()


@pytest.mark.parametrize("tb", DEPTHS)
def test_tblock_mode_is_used(tb):
    """The solves above do run temporally blocked (plan mode 3), at either depth."""
    op = _lat(300, 40, 1.0, 13)
    with kpm.launch_settings(small=0, tblock=tb):
        h = kpm.Hamiltonian(op, 4.2, 0.0, kpm.F64)
        s = kpm.Solve(h, 20, 8, wl.VEC_RADEMACHER, 1, 0)
        mode = kpm.lib().kpm_solve_mode(s._s)
        s.close()
        h.free()
    assert mode == 3
