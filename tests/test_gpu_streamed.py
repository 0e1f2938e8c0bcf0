"""FP32 3D spin solves whose vectors stream from HBM take shorter march segments on a quarter of the
blocks (more work items per block).  Streaming is forced here on lattices small enough for the
oracle: the vectors are bitwise those of the cached plan, so the moments differ from it only by the
order in which the dot partials are summed, and they match the oracle to the FP32 bar."""
import numpy as np
import pytest

import oracle
import paper_1105_5481_amd as kpm
from paper_1105_5481_amd import workloads as wl
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("L,R,M,max_blocks", [(40, 32, 64, None), (33, 20, 41, 64), (24, 7, 30, 8)])
def test_streamed_spin_plan_matches_cached_and_oracle(L, R, M, max_blocks):
    op = wl.spin_cubic_lattice(L, seed=300 + L)
    lo, hi = gu.oracle_bounds(op)
    a, b = oracle.scale_from_bounds(lo, hi, 0.01)
    with kpm.launch_settings(streaming=1, max_blocks=max_blocks):
        streamed = gu.gpu_moments(op, a, b, kpm.F32, M, R, wl.VEC_PHASE, seed=17)
    with kpm.launch_settings(streaming=0):
        cached = gu.gpu_moments(op, a, b, kpm.F32, M, R, wl.VEC_PHASE, seed=17)
    ref = gu.oracle_moments(op, a, b, M, R, wl.VEC_PHASE, 17)
    print(f"  L={L} R={R}: streamed vs cached {np.abs(streamed - cached).max():.2e}, "
          f"vs oracle {np.abs(streamed - ref).max():.2e}")
    assert np.abs(streamed - cached).max() <= 1e-12
    gu.assert_fp32(streamed, ref, f"streamed spin plan L={L}")
