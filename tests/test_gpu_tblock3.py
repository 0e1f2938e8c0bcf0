"""Two recursion steps per pass on 3D lattices (chunk-major vectors, row tiles of whole planes or
with halo rows, segments of planes along z): the vectors are bitwise those of the one-step
recursion, so FP64 moments match the oracle to the usual bar and both precisions match the one-step
march kernels.  Odd step counts and chunk sizes exercise the single-step passes; plane sizes above
one tile exercise the halo rows, ragged last tiles and segments; extents 1 and 2 the slot rules."""
import numpy as np
import pytest

import oracle
import paper_1105_5481_amd as kpm
from paper_1105_5481_amd import workloads as wl
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu


def _cube(L, W, seed, spin):
    Lx, Ly, Lz = L
    N = Lx * Ly * Lz
    onsite = wl.anderson_onsite(N, W, seed) if W > 0 else None
    if spin:
        th, ph = wl.spins_uniform(N, seed)
        return wl.Lattice(dim=3, L=(Lx, Ly, Lz), t=1.0, hop=wl.HOP_SPIN, onsite=onsite, spinor=wl.spinor_of(th, ph),
                          theta=th, phi=ph)
    return wl.Lattice(dim=3, L=(Lx, Ly, Lz), t=1.0, onsite=onsite)


CASES = [  # (extents, W, spin, R, vector kind, M)
    ((10, 10, 10), 0.0, False, 4, wl.VEC_RADEMACHER, 64),   # the paper's cube: one tile per plane
    ((12, 10, 6), 1.0, True, 3, wl.VEC_PHASE, 41),          # odd M: a single step at the end
    ((48, 48, 20), 0.5, True, 4, wl.VEC_PHASE, 30),         # 2304 sites per plane: two row tiles, halo rows
    ((64, 40, 9), 1.0, False, 3, wl.VEC_RADEMACHER, 33),    # two row tiles of 20 rows
    ((150, 7, 5), 1.0, False, 2, wl.VEC_PHASE, 26),         # row tiles of 2, 2, 2 and 1 rows
    ((2, 3, 4), 1.0, True, 2, wl.VEC_PHASE, 20),            # extents 2: wrapped slots kept
    ((5, 1, 7), 0.7, False, 3, wl.VEC_RADEMACHER, 17),      # extent 1: self-loop slots
    ((16, 16, 33), 1.0, True, 9, wl.VEC_PHASE, 50),         # C = 5 (FP32) chunks, several segments
]


def _mode(op, prec, M, R, vec, **kw):
    with kpm.launch_settings(small=0, **kw):
        h = kpm.Hamiltonian(op, 6.5, 0.0, prec)
        s = kpm.Solve(h, M, R, vec, 1, 0)
        m = kpm.lib().kpm_solve_mode(s._s)
        s.close()
        h.free()
    return m


@pytest.mark.parametrize("prec", [kpm.F64, kpm.F32], ids=["f64", "f32"])
@pytest.mark.parametrize("case", CASES, ids=lambda c: "x".join(map(str, c[0])) + ("-spin" if c[2] else "-real"))
def test_tb3_matches_oracle_and_one_step(case, prec):
    L, W, spin, R, vec, M = case
    op = _cube(L, W, sum(L) + 7, spin)
    assert _mode(op, prec, M, R, vec, tblock=-1, tb3=1) == 4
    assert _mode(op, prec, M, R, vec, tblock=0) == 1
    lo, hi = gu.oracle_bounds(op)
    a, b = oracle.scale_from_bounds(lo, hi, 0.01)
    with kpm.launch_settings(small=0, tblock=-1, tb3=1):
        got = gu.gpu_moments(op, a, b, prec, M, R, vec, seed=8, instance=2)
    with kpm.launch_settings(small=0, tblock=0):
        one = gu.gpu_moments(op, a, b, prec, M, R, vec, seed=8, instance=2)
    ref = gu.oracle_moments(op, a, b, M, R, vec, 8, 2)
    print(f"  {L}: two-step vs one-step {np.abs(got - one).max():.2e}, vs oracle {np.abs(got - ref).max():.2e}")
    if prec == kpm.F64:
        gu.assert_fp64(got, ref, "3D two-step passes")
        assert np.abs(got - one).max() <= 1e-15
    else:
        gu.assert_fp32(got, ref, "3D two-step passes")
        assert np.abs(got - one).max() <= 1e-12


@pytest.mark.parametrize("chunks", [[1, 1, 3, 2, 5, 100], [2, 100], [7, 100]])
def test_tb3_chunked_advance(chunks):
    """Single-step and two-step passes in any order keep the four buffers and the dots consistent."""
    op = _cube((48, 48, 20), 1.0, 31, True)
    lo, hi = gu.oracle_bounds(op)
    a, b = oracle.scale_from_bounds(lo, hi, 0.01)
    M, R = 37, 3
    with kpm.launch_settings(small=0, tblock=-1, tb3=1):
        h = kpm.Hamiltonian(op, a, b, kpm.F64)
        s = kpm.Solve(h, M, R, wl.VEC_PHASE, 3, 0)
        assert kpm.lib().kpm_solve_mode(s._s) == 4
        for c in chunks:
            if s.remaining == 0:
                break
            s.advance(c)
        mu = s.finish().cpu().numpy()
        s.close()
        h.free()
    ref = gu.oracle_moments(op, a, b, M, R, wl.VEC_PHASE, 3)
    gu.assert_fp64(mu, ref, f"chunks {chunks}")


def test_tb3_in_a_dynamic_batch_beside_2d_and_csr():
    """3D two-step members share launches with 2D blocked, one-step and CSR members of a dynamic
    batch; every result equals the same solve run alone, bitwise."""
    ops = [_cube((48, 48, 20), 1.0, 41, True), _cube((10, 10, 10), 0.0, 42, False), _cube((16, 16, 33), 1.0, 43, True),
           wl.Lattice(dim=2, L=(300, 40, 1), t=1.0, onsite=wl.anderson_onsite(12000, 1.0, 44)),
           wl.lattice_to_csr(wl.square_lattice(40, W=1.0, seed=45))]
    Ms = [33, 64, 21, 40, 30]
    Rs = [3, 4, 9, 8, 5]
    vecs = [wl.VEC_PHASE, wl.VEC_RADEMACHER, wl.VEC_PHASE, wl.VEC_RADEMACHER, wl.VEC_PHASE]
    with kpm.launch_settings(small=0, tblock=-1, tb3=1):
        hs, ss = [], []
        for k, op in enumerate(ops):
            lo, hi = gu.oracle_bounds(op)
            a, b = oracle.scale_from_bounds(lo, hi, 0.01)
            h = kpm.Hamiltonian(op, a, b, kpm.F32)
            hs.append(h)
            ss.append(kpm.Solve(h, Ms[k], Rs[k], vecs[k], 50 + k, k))
        assert [kpm.lib().kpm_solve_mode(s._s) for s in ss][:4] == [4, 4, 4, 3]
        batch = kpm.Batch(capacity=8)
        for s in ss:
            batch.add(s)
        q = 0
        while any(s.remaining > 0 for s in ss):
            batch.advance([5, 16, 3][q % 3])
            q += 1
        outs = []
        for s in ss:
            batch.remove(s)
            outs.append(s.finish().cpu().numpy())
            s.close()
        batch.free()
        solo = [kpm.moments(h, Ms[k], Rs[k], vecs[k], 50 + k, k).cpu().numpy() for k, h in enumerate(hs)]
    for k, (mu, one) in enumerate(zip(outs, solo)):
        assert np.array_equal(mu, one), (k, float(np.abs(mu - one).max()))
        ref = gu.oracle_moments(ops[k], hs[k].a, hs[k].b, Ms[k], Rs[k], vecs[k], 50 + k, k)
        gu.assert_fp32(mu, ref, f"batched member {k}")
    for h in hs:
        h.free()
