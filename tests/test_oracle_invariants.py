"""Invariants of the moments, the two moment formulas, and the double-double accumulation."""
from fractions import Fraction

import numpy as np
import pytest

from paper_1105_5481_amd import workloads as wl
from tests import _ref


def test_mu0_is_exactly_one_for_pm1(oracle_mod):
    lat = wl.square_lattice(20, W=1.0, seed=4)
    mu = oracle_mod.moments_lattice(2, lat.L, 1.0, 5.0, 0.1, 64, 6, vec_kind=0, seed=9, onsite=lat.onsite)
    assert mu[0] == 1.0
    assert np.abs(mu).max() <= 1.0


def test_moments_bounded_by_one(oracle_mod):
    lat = wl.spin_cubic_lattice(8, seed=2)
    mu = oracle_mod.moments_lattice(3, lat.L, 1.0, 6.0 / 0.99, 0.0, 300, 4, vec_kind=1, seed=1, hop=1,
                                    spinor=lat.spinor)
    assert abs(mu[0] - 1.0) < 1e-15
    assert np.abs(mu).max() <= 1.0 + 1e-15


@pytest.mark.parametrize("L", [(8, 8), (6, 4, 10)])
def test_odd_moments_vanish_on_bipartite_lattice(oracle_mod, L):
    """A unit vector on a bipartite lattice with no diagonal and b = 0: r_n lives on one
    sublattice, so every odd moment is exactly zero (also through the doubling identity)."""
    muB, muA = oracle_mod.moments_lattice(len(L), L, 1.0, 2.0 * len(L) / 0.99, 0.0, 101, 3, vec_kind=2,
                                          formula_a=True)
    assert np.all(muB[1::2] == 0.0)
    assert np.all(muA[1::2] == 0.0)


@pytest.mark.parametrize("vec", [0, 1])
def test_formula_a_equals_formula_b(oracle_mod, vec):
    """Eq. (munr) directly (M-1 products) vs the doubling identities (M/2 products)."""
    lat = wl.square_lattice(24, W=2.0, seed=8)
    for M in (1, 2, 3, 64, 65):
        muB, muA = oracle_mod.moments_lattice(2, lat.L, 1.0, 6.1, -0.05, M, 5, vec_kind=vec, seed=3,
                                              onsite=lat.onsite, formula_a=True)
        assert np.abs(muA - muB).max() < 1e-13, M


def test_prefix_consistency(oracle_mod):
    """Moments do not depend on how many are requested."""
    lat = wl.square_lattice(16, W=1.0, seed=1)
    m_long = oracle_mod.moments_lattice(2, lat.L, 1.0, 5.0, 0.0, 200, 3, seed=2, onsite=lat.onsite)
    for M in (1, 2, 7, 64, 199):
        m = oracle_mod.moments_lattice(2, lat.L, 1.0, 5.0, 0.0, M, 3, seed=2, onsite=lat.onsite)
        assert np.array_equal(m, m_long[:M])


def test_statistical_error_of_estimator(oracle_mod):
    """The estimator's mean over independent instances approaches the exact trace (Sec. II-A),
    with a spread of order 1/sqrt(N R)."""
    L = (6, 6)
    onsite = wl.anderson_onsite(36, 2.0, 17)
    H = _ref.clean_lattice_dense(L) + np.diag(onsite)
    a, b = 7.0, 0.0
    M = 12
    exact = _ref.exact_moments_from_eigh((H - b * np.eye(36)) / a, M)
    est = np.array([oracle_mod.moments_lattice(2, L, 1.0, a, b, M, 4, vec_kind=0, seed=5, instance=s,
                                               onsite=onsite) for s in range(200)])
    err = est.mean(axis=0) - exact
    sem = est.std(axis=0) / np.sqrt(len(est))
    assert np.all(np.abs(err[1:]) < 5 * sem[1:] + 1e-12)
    assert np.all(est.std(axis=0)[1:] < 3.0 / np.sqrt(36 * 4))


def test_double_double_dots_are_exact(oracle_mod):
    """<r_0|r_0> for phase vectors, accumulated in double-double, equals the exact rational sum
    of the squares of the same doubles to far below one unit in the last place, and
    mu_0 is its correctly rounded quotient."""
    N, R, seed = 3000, 3, 31
    X = oracle_mod.start_vectors(1, seed, 0, N, R)
    exact = Fraction(0)
    for v in X.ravel():
        exact += Fraction(v.real) ** 2 + Fraction(v.imag) ** 2
    mu, dots = oracle_mod.moments_lattice(2, (50, 60), 1.0, 5.0, 0.0, 3, R, vec_kind=1, seed=seed,
                                          return_dots=True)
    got = Fraction(dots[0, 0, 0]) + Fraction(dots[0, 0, 1])
    assert abs(got - exact) < Fraction(1, 10**28)
    assert mu[0] == float(exact / (N * R))
    # mu_2 = (2 S_11 - S_00) / (N R), formed in double-double then rounded once
    s11 = Fraction(dots[1, 0, 0]) + Fraction(dots[1, 0, 1])
    assert abs(Fraction(mu[2]) - (2 * s11 - exact) / (N * R)) <= Fraction(abs(mu[2])) * Fraction(1, 2**52)
