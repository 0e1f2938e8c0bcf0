"""Vector blocks of 4 GiB and more take the 64-bit-offset kernel instantiations: checked against
the oracle on the first moments of lattices whose vector block is exactly 2^32 bytes."""
import numpy as np
import pytest

import oracle
import paper_1105_5481_amd as kpm
from paper_1105_5481_amd import workloads as wl
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu

M = 6   # three recursion steps: one pass of three, or a pair and a single step, with temporal blocking


@pytest.mark.parametrize("tblock", [-1, 1, 0])
def test_wide_2d_fp64(tblock):
    """4096^2 sites x 32 real FP64 vectors = 2^32 bytes per vector block."""
    op = wl.square_lattice(4096, t=1.0, W=1.0, seed=21)
    lo, hi = gu.oracle_bounds(op)
    a, b = oracle.scale_from_bounds(lo, hi, 0.01)
    with kpm.launch_settings(tblock=tblock):
        mu = gu.gpu_moments(op, a, b, kpm.F64, M, 32, wl.VEC_RADEMACHER, seed=3)
    ref = gu.oracle_moments(op, a, b, M, 32, wl.VEC_RADEMACHER, 3)
    gu.assert_fp64(mu, ref, f"wide 2D tblock={tblock}")


def test_wide_3d_spin_c64():
    """256^3 sites x 32 complex64 vectors = 2^32 bytes per vector block."""
    op = wl.spin_cubic_lattice(256, seed=22)
    lo, hi = gu.oracle_bounds(op)
    a, b = oracle.scale_from_bounds(lo, hi, 0.01)
    mu = gu.gpu_moments(op, a, b, kpm.F32, M, 32, wl.VEC_PHASE, seed=4)
    ref = gu.oracle_moments(op, a, b, M, 32, wl.VEC_PHASE, 4)
    gu.assert_fp32(mu, ref, "wide 3D spin c64")


def test_wide_2d_spin_c64_tblock():
    """4096^2 spin sites x 32 complex64 vectors = 2^32 bytes per vector block, temporally blocked
    at the default depth (a four-step pass and a single step)."""
    L = 4096
    theta, phi = wl.spins_uniform(L * L, 23)
    op = wl.Lattice(dim=2, L=(L, L, 1), t=1.0, hop=wl.HOP_SPIN, spinor=wl.spinor_of(theta, phi),
                    theta=theta, phi=phi)
    lo, hi = gu.oracle_bounds(op)
    a, b = oracle.scale_from_bounds(lo, hi, 0.01)
    with kpm.launch_settings(tblock=-1, small=0):
        h = kpm.Hamiltonian(op, a, b, kpm.F32)
        s = kpm.Solve(h, 10, 32, wl.VEC_PHASE, 5, 0)
        mode = kpm.lib().kpm_solve_mode(s._s)
        s.advance(100)
        mu = s.finish().cpu().numpy()
        s.close()
        h.free()
    assert mode == 3
    ref = gu.oracle_moments(op, a, b, 10, 32, wl.VEC_PHASE, 5)
    gu.assert_fp32(mu, ref, "wide 2D spin c64, temporal blocking")
