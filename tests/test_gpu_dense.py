"""Dense-H recursion on the matrix cores against the oracle and against the stencil path.

The dense products sum their terms in a different order (and with fused multiply-adds) than the
oracle's row loop, so agreement is to rounding, not bitwise: each step's products carry relative
errors of a few ulp that the (stable) Chebyshev recursion passes on linearly in n; the tolerance
below, |d mu_n| <= 1e-11, is far above that and far below any structural error."""
import numpy as np
import pytest

import oracle
import paper_1105_5481_amd as kpm
from paper_1105_5481_amd import workloads as wl
from tests import _ref
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu

TOL = 1e-11


def _dense_csr(H):
    D = H.shape[0]
    return wl.CSR(n=D, row_ptr=(np.arange(D + 1) * D).astype(np.int64), col=np.tile(np.arange(D), D).astype(np.int32),
                  val_re=np.ascontiguousarray(H.reshape(-1)))


def _goe(D, seed):
    g = np.random.default_rng(seed)
    X = g.normal(size=(D, D)) / np.sqrt(2 * D)
    return X + X.T


def test_e1_lattice_dense_equals_oracle_and_stencil():
    """The paper's E1 matrix: the 10x10x10 cubic lattice with zero diagonal and -1 hopping (D = 1000),
    as a dense matrix."""
    import torch
    op = wl.cubic_lattice(10, t=1.0, W=0.0, seed=1)
    H = _ref.clean_lattice_dense((10, 10, 10), t=1.0)
    lo, hi = gu.oracle_bounds(op)
    a, b = oracle.scale_from_bounds(lo, hi, 0.01)
    M, R, seed = 128, 14, 3
    mu = kpm.dense_moments(torch.tensor(H, device="cuda"), a, b, M, R, wl.VEC_RADEMACHER, seed, 0).cpu().numpy()
    ref = gu.oracle_moments(op, a, b, M, R, wl.VEC_RADEMACHER, seed, 0)
    sten = gu.gpu_moments(op, a, b, kpm.F64, M, R, wl.VEC_RADEMACHER, seed, 0)
    print(f"  E1 dense vs oracle {np.abs(mu - ref).max():.2e}, vs stencil {np.abs(mu - sten).max():.2e}")
    assert np.abs(mu - ref).max() <= TOL
    assert np.abs(mu - sten).max() <= TOL


# (2048, 2048, 6): 1024 output blocks, so the product runs on 64 x 64 blocks; the others on 64 x 32
@pytest.mark.parametrize("D,R,M", [(300, 70, 101), (64, 1, 40), (129, 65, 64), (100, 37, 77), (128, 48, 300),
                                   (2048, 2048, 6)])
def test_random_dense_matches_oracle(D, R, M):
    import torch
    H = _goe(D, D + R)
    lam = np.linalg.eigvalsh(H)
    a, b = oracle.scale_from_bounds(lam[0], lam[-1], 0.05)
    mu = kpm.dense_moments(torch.tensor(H, device="cuda"), a, b, M, R, wl.VEC_RADEMACHER, 7, 2).cpu().numpy()
    c = _dense_csr(H)
    ref = oracle.moments_csr(c.row_ptr, c.col, c.val_re, None, a, b, M, R, wl.VEC_RADEMACHER, 7, 2)
    print(f"  GOE D={D} R={R} M={M}: max |d mu| {np.abs(mu - ref).max():.2e}")
    assert np.abs(mu - ref).max() <= TOL


def test_unit_vectors_give_exact_trace():
    """R = D unit vectors: the exact moments Tr T_n(H~)/D, from a dense eigendecomposition."""
    import torch
    D, M = 90, 64
    H = _goe(D, 11)
    lam = np.linalg.eigvalsh(H)
    a, b = oracle.scale_from_bounds(lam[0], lam[-1], 0.02)
    mu = kpm.dense_moments(torch.tensor(H, device="cuda"), a, b, M, D, wl.VEC_UNIT, 0, 0).cpu().numpy()
    x = (lam - b) / a
    exact = np.array([np.mean(_ref.cheb_T(n, x)) for n in range(M)])
    assert np.abs(mu - exact).max() < 1e-12


def test_complex_vectors_rejected():
    import torch
    H = torch.zeros((8, 8), dtype=torch.float64, device="cuda")
    with pytest.raises(kpm.KPMError):
        kpm.dense_moments(H, 1.0, 0.0, 16, 2, wl.VEC_PHASE)


@pytest.mark.parametrize("D", [16, 72, 128])
def test_on_chip_and_tiled_kernels_agree(D):
    """D <= 128 runs the whole recursion in one launch with H~ in LDS; the tiled product kernel
    (forced with small=0) computes the same moments."""
    import torch
    H = torch.tensor(_goe(D, 3 * D), device="cuda")
    on_chip = kpm.dense_moments(H, 2.2, 0.0, 200, 50, wl.VEC_RADEMACHER, 4, 1).cpu().numpy()
    with kpm.launch_settings(small=0):
        tiled = kpm.dense_moments(H, 2.2, 0.0, 200, 50, wl.VEC_RADEMACHER, 4, 1).cpu().numpy()
    assert np.abs(on_chip - tiled).max() <= TOL
