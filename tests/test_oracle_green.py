"""Pin the oracle's Green's function.

* Single level: the exact moments of a state at x0 are mu_n = T_n(x0) = Re(w^n), w = e^{i phi0}.
  For a kernel that is a combination of geometric sequences (none: g_n = 1; Lorentz:
  sinh(lam (1 - n/M)) = (e^lam r1^n - e^-lam r2^n)/2 with r1 = e^{-lam/M}, r2 = e^{lam/M}), the sum
  sum_n g_n mu_n e^{-i n theta} is a handful of finite geometric series with closed forms, evaluated
  here without any per-n loop.
* Im G = -pi rho: the imaginary part equals the oracle's DoS (Eq. (fKPM)) with the same kernel.
* Lattice: the Lorentz-broadened Green's function of a site approaches the resolvent
  <i|(omega + i eta - H)^{-1}|i> computed from a dense eigendecomposition.
"""
import numpy as np
import pytest

from paper_1105_5481_amd import workloads as wl
from tests import _ref


def _geom(q, M):
    """sum_{n=0}^{M-1} q^n for complex q != 1."""
    return (1.0 - q ** M) / (1.0 - q)


def _closed_single_level(x0, M, K, kernel, lam):
    phi0 = np.arccos(x0)
    theta = np.pi * (np.arange(K) + 0.5) / K
    z = np.exp(-1j * theta)
    w = np.exp(1j * phi0)

    def S(r):   # sum_n r^n T_n(x0) z^n = (S(w r z) + S(r z / w)) / 2
        return 0.5 * (_geom(w * r * z, M) + _geom(r * z / w, M))

    if kernel == 0:
        tot = S(1.0)
    else:
        r1, r2 = np.exp(-lam / M), np.exp(lam / M)
        tot = (np.exp(lam) * S(r1) - np.exp(-lam) * S(r2)) / (2.0 * np.sinh(lam))
    # sum_n (2 - delta_n0) g_n mu_n e^{-i n theta} = 2 tot - g_0 mu_0
    series = 2.0 * tot - 1.0
    return -1j * series / np.sin(theta)


@pytest.mark.parametrize("kernel,lam", [(0, 0.0), (2, 4.0), (2, 1.5)])
@pytest.mark.parametrize("x0", [0.3, -0.71, 0.05])
def test_single_level_closed_form(oracle_mod, kernel, lam, x0):
    M, K = 257, 600
    mu = np.cos(np.arange(M) * np.arccos(x0))
    om, G = oracle_mod.green(mu, K, 1.0, 0.0, kernel, lam)
    ref = _closed_single_level(x0, M, K, kernel, lam)
    assert np.max(np.abs(G - ref)) < 1e-9 * np.max(np.abs(ref))


@pytest.mark.parametrize("kernel", [1, 2])
def test_imaginary_part_is_minus_pi_rho(oracle_mod, kernel):
    g = np.random.default_rng(4)
    M, K, a, b = 128, 300, 2.5, -0.3
    mu = g.normal(size=M) / (1 + np.arange(M))
    mu[0] = 1.0
    om, G = oracle_mod.green(mu, K, a, b, kernel, 4.0)
    if kernel == 1:
        om2, rho = oracle_mod.dos(mu, K, a, b, use_jackson=True)
    else:   # the DoS with the Lorentz kernel written from Eq. (fKPM) directly
        theta, x = oracle_mod.chebyshev_points(K)
        gn = oracle_mod.lorentz(M, 4.0)
        T = np.cos(np.outer(np.arange(M), theta))
        f = (gn[0] * mu[0] + 2 * (gn[1:, None] * mu[1:, None] * T[1:]).sum(axis=0)) / (np.pi * np.sin(theta))
        om2, rho = a * x + b, f / a
    assert np.allclose(om, om2, rtol=0, atol=1e-14)
    assert np.max(np.abs(-G.imag / np.pi - rho)) < 1e-12 * np.max(np.abs(rho))


def test_lattice_site_green_approaches_resolvent(oracle_mod):
    """Site 0 of a 12x12 Anderson lattice: the exact unit-vector moments from the oracle's recursion,
    Lorentz kernel with lam = 4 and M = 2048; away from the band edges the result is within a few
    percent of the resolvent with eta = lam/M in the x variable (times sqrt(1-x^2))."""
    op = wl.square_lattice(12, t=1.0, W=1.0, seed=9)
    H = _ref.clean_lattice_dense((12, 12)) + np.diag(op.onsite)
    E, V = np.linalg.eigh(H)
    a, b = (E[-1] - E[0]) / 1.9, (E[-1] + E[0]) / 2
    M, K, lam = 2048, 400, 4.0
    mu = oracle_mod.moments_lattice(2, (12, 12), 1.0, a, b, M, 1, vec_kind=oracle_mod.VEC_UNIT, instance=0,
                                    onsite=op.onsite)
    om, G = oracle_mod.green(mu, K, a, b, 2, lam)
    x = (om - b) / a
    eta = lam / M * np.sqrt(1 - x ** 2) * a
    w0 = np.abs(V[0]) ** 2
    res = (w0[None, :] / (om[:, None] + 1j * eta[:, None] - E[None, :])).sum(axis=1)
    inner = np.abs(x) < 0.8
    rel = np.abs(G[inner] - res[inner]) / np.abs(res[inner])
    assert np.median(rel) < 0.05
