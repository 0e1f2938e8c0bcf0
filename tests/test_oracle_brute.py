"""Pin the oracle's recursion and both moment formulas to dense eigendecomposition.

For tiny lattices the exact moments mu_n = Tr T_n(H~)/N (Eq. (DoStr)) and the
stochastic estimator for the same start vectors (Eq. (munr)) are computed here
from numpy.linalg.eigh of a dense H assembled independently of the oracle.
"""
import numpy as np
import pytest

from paper_1105_5481_amd import workloads as wl
from tests import _ref

TOL = 1e-12


def _scaled(H, a, b):
    return (H - b * np.eye(H.shape[0])) / a


def _lattice_cases():
    cases = []
    # 2D bipartite with disorder, 2D odd (not bipartite), 3D box, 2D with a self-loop axis
    for L, W, seed in [((4, 4), 1.0, 5), ((5, 3), 2.0, 6), ((3, 4, 5), 1.5, 7), ((6, 1), 0.5, 8)]:
        dim = len(L)
        N = int(np.prod(L))
        onsite = wl.anderson_onsite(N, W, seed)
        H = _ref.clean_lattice_dense(L, t=1.3) + np.diag(onsite)
        cases.append(("real", dim, L, 1.3, 0, onsite, None, H))
    # spin hopping, 3D and 2D
    for L, seed in [((3, 3, 4), 11), ((4, 5), 12)]:
        N = int(np.prod(L))
        th, ph = wl.spins_uniform(N, seed)
        H = _ref.spin_lattice_dense(L, th, ph, t=0.9)
        cases.append(("spin", len(L), L, 0.9, 1, None, wl.spinor_of(th, ph), H))
    return cases


@pytest.mark.parametrize("case", _lattice_cases(), ids=lambda c: f"{c[0]}-{'x'.join(map(str, c[2]))}")
def test_unit_vectors_give_exact_trace(oracle_mod, case):
    kind, dim, L, t, hop, onsite, spinor, H = case
    N = H.shape[0]
    lo, hi = oracle_mod.gershgorin_lattice(dim, L, t, hop, onsite, spinor)
    a, b = oracle_mod.scale_from_bounds(lo, hi, 0.05)
    M = 40
    exact = _ref.exact_moments_from_eigh(_scaled(H, a, b), M)
    muB, muA = oracle_mod.moments_lattice(dim, L, t, a, b, M, N, vec_kind=2, hop=hop, onsite=onsite,
                                          spinor=spinor, formula_a=True)
    assert np.abs(muB - exact).max() < TOL
    assert np.abs(muA - exact).max() < TOL


@pytest.mark.parametrize("vec", [0, 1])
@pytest.mark.parametrize("case", _lattice_cases(), ids=lambda c: f"{c[0]}-{'x'.join(map(str, c[2]))}")
def test_random_vectors_match_eigh_estimator(oracle_mod, case, vec):
    kind, dim, L, t, hop, onsite, spinor, H = case
    N = H.shape[0]
    lo, hi = oracle_mod.gershgorin_lattice(dim, L, t, hop, onsite, spinor)
    a, b = oracle_mod.scale_from_bounds(lo, hi, 0.05)
    M, R, seed, inst = 33, 5, 424242, 2
    X = _ref.start_vectors_numpy(vec, seed, inst, N, R)
    ref = _ref.estimator_from_eigh(_scaled(H, a, b), X, M)
    muB, muA = oracle_mod.moments_lattice(dim, L, t, a, b, M, R, vec_kind=vec, seed=seed, instance=inst,
                                          hop=hop, onsite=onsite, spinor=spinor, formula_a=True)
    assert np.abs(muB - ref).max() < TOL
    assert np.abs(muA - ref).max() < TOL


@pytest.mark.parametrize("complex_values", [False, True])
def test_csr_matches_eigh(oracle_mod, complex_values):
    csr = wl.random_hermitian_csr(48, 6, seed=3, complex_values=complex_values)
    H = _ref.csr_dense(csr)
    assert np.abs(H - H.conj().T).max() == 0.0
    lo, hi = oracle_mod.gershgorin_csr(csr.row_ptr, csr.col, csr.val_re, csr.val_im)
    E = np.linalg.eigvalsh(H)
    assert lo <= E.min() and E.max() <= hi
    a, b = oracle_mod.scale_from_bounds(lo, hi, 0.02)
    M = 30
    exact = _ref.exact_moments_from_eigh(_scaled(H, a, b), M)
    mu = oracle_mod.moments_csr(csr.row_ptr, csr.col, csr.val_re, csr.val_im, a, b, M, csr.n, vec_kind=2)
    assert np.abs(mu - exact).max() < TOL
    X = _ref.start_vectors_numpy(1, 77, 0, csr.n, 3)
    ref = _ref.estimator_from_eigh(_scaled(H, a, b), X, M)
    muB, muA = oracle_mod.moments_csr(csr.row_ptr, csr.col, csr.val_re, csr.val_im, a, b, M, 3,
                                      vec_kind=1, seed=77, formula_a=True)
    assert np.abs(muB - ref).max() < TOL
    assert np.abs(muA - ref).max() < TOL


def test_lattice_as_csr_gives_same_moments(oracle_mod):
    """The lattice path and the CSR path of the oracle agree on the same operator
    (the CSR is assembled by the input module from the hopping formula)."""
    lat = wl.spin_cubic_lattice(4, seed=21)
    csr = wl.lattice_to_csr(lat)
    a, b = 6.2, 0.1
    m1 = oracle_mod.moments_lattice(3, lat.L, lat.t, a, b, 50, 3, vec_kind=1, seed=5, hop=1,
                                    spinor=lat.spinor)
    m2 = oracle_mod.moments_csr(csr.row_ptr, csr.col, csr.val_re, csr.val_im, a, b, 50, 3,
                                vec_kind=1, seed=5)
    assert np.abs(m1 - m2).max() < 1e-13


def _discs(H):
    """Gershgorin bounds written from a dense matrix: min/max over rows of Re H_ii -/+ sum_{j!=i} |H_ij|,
    with |.| the complex modulus."""
    off = np.abs(H).sum(axis=1) - np.abs(np.diag(H))
    return (np.diag(H).real - off).min(), (np.diag(H).real + off).max()


@pytest.mark.parametrize("case", _lattice_cases(), ids=lambda c: f"{c[0]}-{'x'.join(map(str, c[2]))}")
def test_gershgorin_contains_spectrum(oracle_mod, case):
    """Real and spin (complex) hopping: the oracle's bounds equal the disc bounds of the dense
    matrix (Sec. II-A, below Eq. (tilde)) and enclose its spectrum.  For complex bonds the radius
    uses the modulus, so a |Re| + |Im| radius would fail the equality."""
    kind, dim, L, t, hop, onsite, spinor, H = case
    lo, hi = oracle_mod.gershgorin_lattice(dim, L, t, hop, onsite, spinor)
    E = np.linalg.eigvalsh(H)
    assert lo <= E.min() + 1e-12 and E.max() <= hi + 1e-12
    if min(L) <= 2:
        # a neighbour slot that wraps onto the site itself counts as an off-diagonal entry (each of
        # the 2 dim slots adds |t| to the radius), where the dense matrix folds it into H_ii
        assert kind == "real"
        assert lo == pytest.approx(onsite.min() - 2 * dim * abs(t), abs=1e-12)
        assert hi == pytest.approx(onsite.max() + 2 * dim * abs(t), abs=1e-12)
        return
    dlo, dhi = _discs(H)
    assert lo == pytest.approx(dlo, abs=1e-12)
    assert hi == pytest.approx(dhi, abs=1e-12)
    if kind == "spin":
        # the pin separates the modulus from the |Re| + |Im| reading
        alt = (np.abs(H.real) + np.abs(H.imag)).sum(axis=1) - np.abs(np.diag(H))
        assert abs((np.diag(H).real - alt).min() - dlo) > 1e-3


@pytest.mark.parametrize("complex_values", [False, True])
def test_gershgorin_csr_equals_dense_discs(oracle_mod, complex_values):
    """CSR input (real and complex entries, Hermitian): the oracle's bounds equal the dense discs."""
    csr = wl.random_hermitian_csr(64, 7, seed=19, complex_values=complex_values)
    H = _ref.csr_dense(csr)
    lo, hi = oracle_mod.gershgorin_csr(csr.row_ptr, csr.col, csr.val_re, csr.val_im)
    dlo, dhi = _discs(H)
    assert lo == pytest.approx(dlo, abs=1e-12)
    assert hi == pytest.approx(dhi, abs=1e-12)
    E = np.linalg.eigvalsh(H)
    assert lo <= E.min() and E.max() <= hi
    if complex_values:
        alt = (np.abs(H.real) + np.abs(H.imag)).sum(axis=1) - np.abs(np.diag(H))
        assert abs((np.diag(H).real - alt).min() - dlo) > 1e-3
