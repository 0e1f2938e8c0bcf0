"""Pin the oracle's DoS reconstruction, Eq. (fKPM), and its Jackson coefficients."""
import mpmath
import numpy as np
import pytest

from tests import _ref


@pytest.mark.parametrize("M", [1, 2, 5, 64, 257, 1024])
def test_jackson_is_normalised_autocorrelation(oracle_mod, M):
    """The Jackson coefficients equal the normalised autocorrelation of the window
    a_nu = sin(pi (nu+1)/(M+1)), nu = 0..M-1 (the positive-kernel construction)."""
    g = oracle_mod.jackson(M)
    a = np.sin(np.pi * (np.arange(M) + 1) / (M + 1))
    ac = np.array([np.dot(a[:M - n], a[n:]) for n in range(M)]) / np.dot(a, a)
    assert np.abs(g - ac).max() < 1e-14
    assert g[0] == pytest.approx(1.0, abs=1e-15)
    assert np.all(np.diff(g) < 0) if M > 1 else True


def test_arcsine_law():
    """mu = (1, 0, 0, ...) is the expansion of f(x) = 1 / (pi sqrt(1 - x^2))."""
    import oracle
    K, a, b = 64, 2.0, 0.5
    om, rho = oracle.dos(np.r_[1.0, np.zeros(9)], K, a, b)
    theta, x = oracle.chebyshev_points(K)
    assert np.allclose(om, a * x + b, rtol=0, atol=1e-15)
    assert np.abs(rho * a * np.pi * np.sqrt(1 - x**2) - 1.0).max() < 1e-12


@pytest.mark.parametrize("K,M", [(16, 20), (1024, 256), (300, 512)])
def test_gauss_chebyshev_normalisation(oracle_mod, K, M):
    """The K-point Gauss-Chebyshev rule integrates T_n exactly for n < 2K, so the quadrature of
    the reconstructed density returns g_0 mu_0 whenever M <= 2K."""
    g = np.random.default_rng(1)
    mu = np.r_[1.0, g.uniform(-0.3, 0.3, M - 1)]
    a, b = 3.0, -1.0
    om, rho = oracle_mod.dos(mu, K, a, b, use_jackson=False)
    theta, x = oracle_mod.chebyshev_points(K)
    integral = np.sum(rho * a * np.sin(theta)) * np.pi / K            # d omega = a dx
    assert integral == pytest.approx(1.0, abs=1e-12)


def test_dct_against_high_precision():
    """Eq. (fKPM) evaluated with 40-digit arithmetic at every grid point."""
    import oracle
    M, K = 23, 17
    g = np.random.default_rng(5)
    mu = np.r_[1.0, g.uniform(-0.5, 0.5, M - 1)]
    om, rho = oracle.dos(mu, K, 1.0, 0.0)
    gj = oracle.jackson(M)
    mpmath.mp.dps = 40
    for k in range(K):
        th = mpmath.pi * (k + mpmath.mpf(1) / 2) / K
        s = gj[0] * mpmath.mpf(mu[0]) + 2 * sum(mpmath.mpf(gj[n]) * mpmath.mpf(mu[n]) * mpmath.cos(n * th)
                                              for n in range(1, M))
        f = s / (mpmath.pi * mpmath.sin(th))
        assert abs(float(f) - rho[k]) < 1e-14 * max(1.0, abs(float(f)))


def test_jackson_dos_of_exact_moments_is_positive(oracle_mod):
    """The Jackson kernel is positive, so the damped expansion of a spectral density is >= 0."""
    L = (8, 8)
    H = _ref.clean_lattice_dense(L) + np.diag(np.random.default_rng(2).uniform(-1, 1, 64))
    a, b = 5.5, 0.0
    mu = _ref.exact_moments_from_eigh(H / a, 128)
    om, rho = oracle_mod.dos(mu, 512, a, b)
    assert rho.min() > -1e-12
    om2, rho2 = oracle_mod.dos(mu, 512, a, b, use_jackson=False)
    assert rho2.min() < -1e-3             # the undamped truncation shows Gibbs oscillations


def test_delta_peak_position_and_width(oracle_mod):
    """A single level x0 has mu_n = T_n(x0); the Jackson-damped expansion peaks at x0 and its
    width shrinks roughly like pi / M (the resolution-vs-truncation trade-off of the paper's
    DoS comparison at N = 256 and 512)."""
    x0 = 0.3
    widths = []
    for M in (256, 512):
        mu = _ref.cheb_T(np.arange(M), x0)
        om, rho = oracle_mod.dos(mu, 8 * M, 1.0, 0.0)
        k = np.argmax(rho)
        assert abs(om[k] - x0) < 2.0 / M
        half = rho > rho[k] / 2
        widths.append(om[half].max() - om[half].min())
    assert 1.6 < widths[0] / widths[1] < 2.4
