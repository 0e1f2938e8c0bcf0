"""Pin the oracle's Philox4x64-10 and start vectors to numpy's independent implementation."""
import numpy as np
import pytest

from tests import _ref


def test_philox_matches_numpy(oracle_mod):
    g = np.random.default_rng(7)
    for _ in range(200):
        ctr = [int(x) for x in g.integers(0, 2**64, size=4, dtype=np.uint64)]
        key = [int(x) for x in g.integers(0, 2**64, size=2, dtype=np.uint64)]
        mine = oracle_mod.philox4x64_10(ctr, key)
        ref = _ref.numpy_philox_block(ctr, key)
        assert (mine == ref).all(), (ctr, key)


def test_philox_edge_counters(oracle_mod):
    for ctr, key in [([0, 0, 0, 0], [0, 0]), ([2**64 - 1] * 4, [2**64 - 1] * 2),
                     ([1, 0, 0, 0], [0, 4]), ([0, 1, 0, 0], [1, 4])]:
        assert (oracle_mod.philox4x64_10(ctr, key) == _ref.numpy_philox_block(ctr, key)).all()


@pytest.mark.parametrize("kind", [0, 1, 2])
def test_start_vectors_match_numpy(oracle_mod, kind):
    N, R, seed, inst = 37, 9, 12345, 3
    mine = oracle_mod.start_vectors(kind, seed, inst, N, R)
    ref = _ref.start_vectors_numpy(kind, seed, inst, N, R)
    assert np.array_equal(mine, ref)


def test_phase_factors_are_roots_of_unity():
    """The half-angle table reproduces exp(2 pi i 2^j / 2^30) to a few ulp (40-digit reference),
    and random phases are uniform on the grid: k/2^30 equals phi/(2 pi) to 1e-14."""
    import mpmath
    mpmath.mp.dps = 40
    for j, (c, s) in enumerate(_ref.phase_factors()):
        t = 2 * mpmath.pi * mpmath.mpf(2) ** j / mpmath.mpf(2) ** 30
        assert abs(c - float(mpmath.cos(t))) < 4e-16 and abs(s - float(mpmath.sin(t))) < 4e-16, j
    g = np.random.default_rng(3)
    for w in g.integers(0, 2**64, 2000, dtype=np.uint64):
        z = _ref.phase_of_word(int(w))
        k = int(w) >> 34
        phi = (np.angle(z) / (2 * np.pi)) % 1.0
        assert abs(abs(z) - 1.0) < 1e-14
        assert min(abs(phi - k / 2**30), 1 - abs(phi - k / 2**30)) < 1e-14


def test_start_vector_statistics(oracle_mod):
    """Mean 0 and unit variance (Sec. II-A): unit modulus exactly for +-1, to rounding for phases."""
    X = oracle_mod.start_vectors(0, 99, 0, 4096, 8)
    assert set(np.unique(X.real)) == {-1.0, 1.0}
    assert abs(X.real.mean()) < 5.0 / np.sqrt(X.size)
    P = oracle_mod.start_vectors(1, 99, 0, 4096, 8)
    assert np.abs(np.abs(P) - 1.0).max() < 1e-14
    assert abs(P.mean()) < 5.0 / np.sqrt(P.size)
    # phases of different (r, i) are uncorrelated: <xi* xi'> ~ 0
    assert abs(np.vdot(P[0], P[1])) / P.shape[1] < 5.0 / np.sqrt(P.shape[1])
