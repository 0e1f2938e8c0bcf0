"""Temporal blocking (several recursion steps per pass) on 2D lattices with real or spin hopping:
the vectors are bitwise those of the one-step recursion, so FP64 moments match the oracle to the
usual bar and both precisions match the one-step path; step counts and chunk sizes that are not
multiples of the pass depth exercise the shorter passes between the deepest ones, and wide sites
(many chunks) the cap of the depth at a quarter of the tile window."""
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
    (260, 20, 1.0, 36, kpm.F32, 50),   # C = 9: a window of 56 sites, 8 of 512 threads idle
    (260, 20, 1.0, 36, kpm.F64, 37),   # C = 18: a window of 28 sites, depth capped at 7
]
DEPTHS = [1, 3, 4, 5, 6]   # KPM_LAUNCH_TBLOCK: steps per pass (1 means two)


def _lat(Lx, Ly, W, seed):
    onsite = wl.anderson_onsite(Lx * Ly, W, seed) if W > 0 else None
    return wl.Lattice(dim=2, L=(Lx, Ly, 1), t=1.0, onsite=onsite)


def _spin_lat(Lx, Ly, W, seed):
    onsite = wl.anderson_onsite(Lx * Ly, W, seed) if W > 0 else None
    theta, phi = wl.spins_uniform(Lx * Ly, seed)
    return wl.Lattice(dim=2, L=(Lx, Ly, 1), t=1.0, hop=wl.HOP_SPIN, onsite=onsite,
                      spinor=wl.spinor_of(theta, phi), theta=theta, phi=phi)


SPIN_CASES = [  # (Lx, Ly, W, R, prec, M, vector kind, spin hopping): chunks per site C -> depth cap 128 / C
    (200, 24, 1.0, 4, kpm.F64, 40, wl.VEC_PHASE, True),      # C = 4
    (96, 20, 0.0, 64, kpm.F32, 31, wl.VEC_PHASE, True),      # C = 32: depth capped at 4
    (40, 12, 0.5, 128, kpm.F32, 13, wl.VEC_PHASE, True),     # C = 64: depth capped at 2
    (300, 18, 1.0, 3, kpm.F32, 26, wl.VEC_RADEMACHER, True),  # C = 2: real vectors, complex operator
    (150, 20, 1.0, 8, kpm.F64, 30, wl.VEC_PHASE, False),     # C = 8: real hopping, complex vectors
    (200, 24, 1.0, 20, kpm.F32, 33, wl.VEC_PHASE, True),     # C = 10: a window of 51 sites
    (200, 24, 0.5, 5, kpm.F64, 29, wl.VEC_PHASE, True),      # C = 5: a window of 102 sites
]


@pytest.mark.parametrize("tb", DEPTHS)
@pytest.mark.parametrize("case", SPIN_CASES,
                         ids=lambda c: f"{'spin' if c[7] else 'real'}{c[0]}x{c[1]}-R{c[3]}-{'f64' if c[4] == 0 else 'f32'}-v{c[6]}")
def test_tblock_complex_matches_oracle_and_one_step(case, tb):
    Lx, Ly, W, R, prec, M, vec, spin = case
    op = (_spin_lat if spin else _lat)(Lx, Ly, W, Lx * Ly + 3)
    lo, hi = gu.oracle_bounds(op)
    a, b = oracle.scale_from_bounds(lo, hi, 0.01)
    with kpm.launch_settings(small=0, tblock=tb):
        h = kpm.Hamiltonian(op, a, b, prec)
        s = kpm.Solve(h, 20, R, vec, 1, 0)
        mode = kpm.lib().kpm_solve_mode(s._s)
        s.close()
        h.free()
        got = gu.gpu_moments(op, a, b, prec, M, R, vec, seed=6)
    assert mode == 3
    with kpm.launch_settings(small=0, tblock=0):
        one = gu.gpu_moments(op, a, b, prec, M, R, vec, seed=6)
    ref = gu.oracle_moments(op, a, b, M, R, vec, 6)
    print(f"  tblock vs one-step {np.abs(got - one).max():.2e}, vs oracle {np.abs(got - ref).max():.2e}")
    if prec == kpm.F64:
        gu.assert_fp64(got, ref, "temporal blocking")
        assert np.abs(got - one).max() <= 1e-15
    else:
        gu.assert_fp32(got, ref, "temporal blocking")
        assert np.abs(got - one).max() <= 1e-12


def test_wide_sites_blocked_through_chunk_groups():
    """128 chunks per site leave a 4-site window for the whole site: too narrow for any halo, so
    without chunk groups the solve takes one step per pass; split into groups of 16 chunks (a
    32-site window within L_x = 40) it is blocked, and its moments equal the one-step path's."""
    op = _spin_lat(40, 12, 0.0, 5)
    modes = {}
    for grp in (0, 8):
        with kpm.launch_settings(small=0, tblock=4, tb_group=grp):
            h = kpm.Hamiltonian(op, 4.5, 0.0, kpm.F32)
            s = kpm.Solve(h, 20, 256, wl.VEC_PHASE, 1, 0)
            modes[grp] = kpm.lib().kpm_solve_mode(s._s)
            s.close()
            h.free()
    assert modes[0] != 3 and modes[8] == 3
    lo, hi = gu.oracle_bounds(op)
    a, b = oracle.scale_from_bounds(lo, hi, 0.01)
    with kpm.launch_settings(small=0, tblock=4, tb_group=8):
        got = gu.gpu_moments(op, a, b, kpm.F32, 20, 256, wl.VEC_PHASE, seed=4)
    with kpm.launch_settings(small=0, tblock=0):
        one = gu.gpu_moments(op, a, b, kpm.F32, 20, 256, wl.VEC_PHASE, seed=4)
    assert np.abs(got - one).max() <= 1e-12


@pytest.mark.parametrize("grp", [0, 4, 8, 16])
def test_chunk_groups_match_oracle(grp):
    """The 2D blocked kernel with the site's chunks split into groups (window of 512 / Cg sites):
    FP64 vectors bitwise those of one-step passes, both precisions against the oracle."""
    op = _spin_lat(300, 24, 1.0, 19)   # R = 64 phase vectors: C = 32 (FP32), 64 (FP64) chunks
    lo, hi = gu.oracle_bounds(op)
    a, b = oracle.scale_from_bounds(lo, hi, 0.01)
    M, R = 45, 64
    ref = gu.oracle_moments(op, a, b, M, R, wl.VEC_PHASE, 12)
    for prec in (kpm.F64, kpm.F32):
        with kpm.launch_settings(small=0, tblock=-1, tb_group=grp):
            h = kpm.Hamiltonian(op, a, b, prec)
            s = kpm.Solve(h, M, R, wl.VEC_PHASE, 12, 0)
            assert kpm.lib().kpm_solve_mode(s._s) == 3
            s.close()
            h.free()
            got = gu.gpu_moments(op, a, b, prec, M, R, wl.VEC_PHASE, seed=12)
        with kpm.launch_settings(small=0, tblock=0):
            one = gu.gpu_moments(op, a, b, prec, M, R, wl.VEC_PHASE, seed=12)
        if prec == kpm.F64:
            gu.assert_fp64(got, ref, f"chunk groups >= {grp}")
            assert np.abs(got - one).max() <= 1e-15
        else:
            gu.assert_fp32(got, ref, f"chunk groups >= {grp}")
            assert np.abs(got - one).max() <= 1e-12


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


@pytest.mark.parametrize("prec,spin,expect", [(kpm.F32, True, True), (kpm.F64, True, True),
                                              (kpm.F32, False, True), (kpm.F64, False, True)])
def test_tblock_default_by_precision_and_hopping(prec, spin, expect):
    """The default (-1) blocks 2D solves of both precisions and hopping kinds."""
    op = (_spin_lat if spin else _lat)(300, 40, 1.0, 17)
    with kpm.launch_settings(small=0, tblock=-1):
        h = kpm.Hamiltonian(op, 4.6, 0.0, prec)
        s = kpm.Solve(h, 20, 8, wl.VEC_PHASE, 1, 0)
        mode = kpm.lib().kpm_solve_mode(s._s)
        s.close()
        h.free()
    assert (mode == 3) == expect


@pytest.mark.parametrize("tb", [-1, 1, 3, 6])
@pytest.mark.parametrize("chunks", [[16], [5, 7, 64], [3, 1, 2, 9]])
def test_tblock_batched_passes_equal_solo(chunks, tb):
    """Temporally blocked solves of different depths, step counts and buffer states share the
    blocked launches of a dynamic batch (a one-step solve beside them): every result equals the
    same solve run alone, bitwise, and the FP64 ones match the oracle."""
    specs = [  # (operator, precision, M, R, vector kind): remainders 0..depth-1 over the chunks
        (_lat(300, 40, 1.0, 21), kpm.F64, 41, 8, wl.VEC_RADEMACHER),
        (_lat(260, 20, 2.0, 22), kpm.F64, 30, 36, wl.VEC_RADEMACHER),
        (_spin_lat(200, 24, 1.0, 23), kpm.F64, 27, 4, wl.VEC_PHASE),
        (_lat(300, 40, 0.5, 24), kpm.F64, 64, 8, wl.VEC_PHASE),
        (wl.spin_cubic_lattice(12, seed=25), kpm.F64, 33, 3, wl.VEC_PHASE),
    ]
    with kpm.launch_settings(small=0, tblock=tb):
        hs, ss, modes = [], [], []
        for k, (op, prec, M, R, vec) in enumerate(specs):
            lo, hi = gu.oracle_bounds(op)
            a, b = oracle.scale_from_bounds(lo, hi, 0.01)
            h = kpm.Hamiltonian(op, a, b, prec)
            hs.append(h)
            s = kpm.Solve(h, M, R, vec, 30 + k, k)
            modes.append(kpm.lib().kpm_solve_mode(s._s))
            ss.append(s)
        assert modes[:4] == [3, 3, 3, 3] and modes[4] != 3
        # one solve joins late, after the others have advanced
        batch = kpm.Batch(capacity=8)
        for s in ss[:-1]:
            batch.add(s)
        q = 0
        while any(s.remaining > 0 for s in ss):
            batch.advance(chunks[q % len(chunks)])
            q += 1
            if q == 1:
                batch.add(ss[-1])
        outs = []
        for s in ss:
            batch.remove(s)
            outs.append(s.finish().cpu().numpy())
            s.close()
        batch.free()
        solo = [kpm.moments(h, M, R, vec, 30 + k, k).cpu().numpy() for k, (h, (_, _, M, R, vec)) in
                enumerate(zip(hs, specs))]
    for k, ((op, prec, M, R, vec), h, mu, one) in enumerate(zip(specs, hs, outs, solo)):
        assert np.array_equal(mu, one), (k, float(np.abs(mu - one).max()))
        ref = gu.oracle_moments(op, h.a, h.b, M, R, vec, 30 + k, k)
        gu.assert_fp64(mu, ref, f"batched blocked solve {k}")
        h.free()
