"""Pin the oracle's Lanczos process and spectral-interval estimate.

* The 1D chain from a site (a CSR ring, unit start vector): alpha_j = 0, beta_0 = sqrt(2) t/a,
  beta_j = t/a until the Krylov space wraps round the ring (a closed form).
* Gauss quadrature: the eigenpairs (theta_i, y_i) of the k x k Lanczos matrix reproduce
  <v_0|T_n(H~)|v_0> = sum_i y_i[0]^2 T_n(theta_i) exactly for n <= 2k - 1, and the left side is
  the oracle's KPM recursion with the same start vector (an independent code path).
* alpha_0, beta_0 from a dense H assembled independently of the oracle.
* Dense spectra: the Ritz values lie inside [lambda_min, lambda_max]; with k = N the extreme
  ones equal them; the padded interval encloses the spectrum and stays inside Gershgorin's.
"""
import numpy as np
import pytest

from paper_1105_5481_amd import workloads as wl
from tests import _ref


def _ring_csr(N, t):
    rows, cols, vals = [], [], []
    for i in range(N):
        for j in ((i - 1) % N, (i + 1) % N):
            rows.append(i); cols.append(j); vals.append(-t)
    order = np.lexsort((cols, rows))
    rows, cols, vals = np.array(rows)[order], np.array(cols)[order], np.array(vals)[order]
    rp = np.searchsorted(rows, np.arange(N + 1))
    return wl.CSR(n=N, row_ptr=rp.astype(np.int64), col=cols.astype(np.int32), val_re=vals.astype(np.float64))


def test_chain_closed_form(oracle_mod):
    N, t, a = 128, 1.7, 3.5
    c = _ring_csr(N, t)
    al, be = oracle_mod.lanczos_csr(c.row_ptr, c.col, c.val_re, None, a, 0.0, 60, vec_kind=oracle_mod.VEC_UNIT,
                                    instance=5)
    assert np.all(np.abs(al) < 1e-14)
    assert abs(be[0] - np.sqrt(2.0) * t / a) < 1e-14
    assert np.max(np.abs(be[1:60] - t / a)) < 1e-13


def _lattice_ops():
    ops = []
    op = wl.square_lattice(6, t=1.2, W=2.0, seed=3)
    ops.append(("square", op, _ref.clean_lattice_dense((6, 6), t=1.2) + np.diag(op.onsite), wl.VEC_RADEMACHER))
    L = (3, 4, 3)
    th, ph = wl.spins_uniform(36, 4)
    op = wl.Lattice(dim=3, L=L, t=0.8, hop=wl.HOP_SPIN, spinor=wl.spinor_of(th, ph))
    ops.append(("spin3d", op, _ref.spin_lattice_dense(L, th, ph, t=0.8), wl.VEC_PHASE))
    c = wl.random_hermitian_csr(30, 4, seed=7)
    ops.append(("csr", c, _ref.csr_dense(c), wl.VEC_PHASE))
    return ops


def _lanczos(oracle_mod, op, a, b, k, vec, seed=9, instance=2):
    if hasattr(op, "row_ptr"):
        return oracle_mod.lanczos_csr(op.row_ptr, op.col, op.val_re, op.val_im, a, b, k, vec, seed, instance)
    return oracle_mod.lanczos_lattice(op.dim, op.L[:op.dim], op.t, a, b, k, vec, seed, instance, hop=op.hop,
                                      onsite=op.onsite, spinor=op.spinor)


def _moments(oracle_mod, op, a, b, M, vec, seed=9, instance=2):
    if hasattr(op, "row_ptr"):
        return oracle_mod.moments_csr(op.row_ptr, op.col, op.val_re, op.val_im, a, b, M, 1, vec, seed, instance)
    return oracle_mod.moments_lattice(op.dim, op.L[:op.dim], op.t, a, b, M, 1, vec, seed, instance, hop=op.hop,
                                      onsite=op.onsite, spinor=op.spinor)


@pytest.mark.parametrize("case", _lattice_ops(), ids=lambda c: c[0])
def test_gauss_quadrature_matches_recursion(oracle_mod, case):
    name, op, H, vec = case
    lo, hi = np.linalg.eigvalsh(H)[[0, -1]]
    a, b = (hi - lo) / 1.9, (hi + lo) / 2
    k = 8
    al, be = _lanczos(oracle_mod, op, a, b, k, vec)
    T = np.diag(al) + np.diag(be[:-1], 1) + np.diag(be[:-1], -1)
    th, Y = np.linalg.eigh(T)
    M = 2 * k
    mu = _moments(oracle_mod, op, a, b, M, vec)
    quad = np.array([np.sum(Y[0] ** 2 * _ref.cheb_T(n, th)) for n in range(M)])
    assert np.max(np.abs(quad - mu)) < 1e-12, name


@pytest.mark.parametrize("case", _lattice_ops(), ids=lambda c: c[0])
def test_first_coefficients_from_dense(oracle_mod, case):
    name, op, H, vec = case
    a, b = 2.5, 0.3
    Ht = (H - b * np.eye(len(H))) / a
    al, be = _lanczos(oracle_mod, op, a, b, 2, vec)
    xi = oracle_mod.start_vectors(vec, 9, 2, len(H), 1)[0]
    v0 = xi / np.linalg.norm(xi)
    u = Ht @ v0
    a0 = np.vdot(v0, u).real
    assert abs(al[0] - a0) < 1e-13
    assert abs(be[0] - np.linalg.norm(u - a0 * v0)) < 1e-13


@pytest.mark.parametrize("case", _lattice_ops(), ids=lambda c: c[0])
def test_bounds_enclose_spectrum(oracle_mod, case):
    name, op, H, vec = case
    lam = np.linalg.eigvalsh(H)
    if hasattr(op, "row_ptr"):
        g = oracle_mod.gershgorin_csr(op.row_ptr, op.col, op.val_re, op.val_im)
    else:
        g = oracle_mod.gershgorin_lattice(op.dim, op.L[:op.dim], op.t, op.hop, op.onsite, op.spinor)
    N = len(H)
    for k in (10, N):
        al, be = _lanczos(oracle_mod, op, 1.0, 0.0, k, vec)
        r = oracle_mod.lanczos_bounds(al, be, 1.0, 0.0, pad=0.005, clamp=g)
        assert lam[0] - 1e-12 <= r["theta_min"] and r["theta_max"] <= lam[-1] + 1e-12
        assert r["e_lo"] <= lam[0] and r["e_hi"] >= lam[-1], (name, k, r, lam[[0, -1]])
        assert g[0] <= r["e_lo"] and r["e_hi"] <= g[1]
        if k == N:
            assert abs(r["theta_min"] - lam[0]) < 1e-10 and abs(r["theta_max"] - lam[-1]) < 1e-10, name


def test_breakdown_truncates(oracle_mod):
    """Start vector in a 2-dimensional invariant subspace: the process stops after 2 steps and the
    Ritz values are exact eigenvalues with zero residual."""
    c = _ring_csr(8, 1.0)
    # a diagonal operator: the unit start vector e_j is an eigenvector
    d = wl.CSR(n=6, row_ptr=np.arange(7, dtype=np.int64), col=np.arange(6, dtype=np.int32),
               val_re=np.array([0.5, -1.0, 2.0, 0.25, -0.75, 1.5]))
    al, be = oracle_mod.lanczos_csr(d.row_ptr, d.col, d.val_re, None, 1.0, 0.0, 5, vec_kind=oracle_mod.VEC_UNIT,
                                    instance=2)
    r = oracle_mod.lanczos_bounds(al, be)
    assert r["m"] == 1 and r["theta_min"] == 2.0 and r["r_max"] == 0.0
    assert r["e_lo"] == 2.0 and r["e_hi"] == 2.0
    al, be = oracle_mod.lanczos_csr(c.row_ptr, c.col, c.val_re, None, 1.0, 0.0, 8, vec_kind=oracle_mod.VEC_UNIT)
    r = oracle_mod.lanczos_bounds(al, be)
    # the ring of 8 seen from a site: 5 distinct eigenvalues 2cos(2 pi q/8) with nonzero weight
    assert r["m"] == 5
    assert abs(r["theta_min"] + 2.0) < 1e-13 and abs(r["theta_max"] - 2.0) < 1e-13


def _numpy_lanczos(Ht, v0, k):
    """The three-term Lanczos process written out in numpy on a dense matrix: returns the basis
    V (N x k), alpha, beta (k each) with H~ V = V T + beta_{k-1} v_k e_{k-1}^T."""
    N = len(v0)
    V = np.zeros((N, k + 1), dtype=complex)
    al, be = np.zeros(k), np.zeros(k)
    V[:, 0] = v0 / np.linalg.norm(v0)
    for j in range(k):
        u = Ht @ V[:, j]
        al[j] = np.vdot(V[:, j], u).real
        w = u - al[j] * V[:, j] - (be[j - 1] * V[:, j - 1] if j > 0 else 0.0)
        be[j] = np.linalg.norm(w)
        V[:, j + 1] = w / be[j]
    return V[:, :k], al, be


@pytest.mark.parametrize("case", _lattice_ops(), ids=lambda c: c[0])
@pytest.mark.parametrize("k", [6, 12])
def test_residual_bound_equals_dense_residual(oracle_mod, case, k):
    """The residual bound r = beta_{m-1} |y_{m-1}| of each extreme Ritz pair (theta, y) is the norm
    ||H~ V y - theta V y|| of its Ritz vector, with V the Lanczos basis built here by a numpy
    Lanczos on the dense matrix from the same start vector (numpy's Philox).  Reading y_0 for
    y_{m-1} would fail: the two differ by far more than the tolerance on these cases."""
    name, op, H, vec = case
    lam = np.linalg.eigvalsh(H)
    a, b = (lam[-1] - lam[0]) / 1.9, (lam[-1] + lam[0]) / 2
    Ht = (H - b * np.eye(len(H))) / a
    al, be = _lanczos(oracle_mod, op, a, b, k, vec)
    r = oracle_mod.lanczos_bounds(al, be, 1.0, 0.0, pad=0.0)
    assert r["m"] == k
    xi = _ref.start_vectors_numpy(vec, 9, 2, len(H), 1)[0]
    V, al_np, be_np = _numpy_lanczos(Ht, xi, k)
    assert np.max(np.abs(al_np - al)) < 1e-12 and np.max(np.abs(be_np - be)) < 1e-12
    T = np.diag(al) + np.diag(be[:-1], 1) + np.diag(be[:-1], -1)
    th, Y = np.linalg.eigh(T)
    for col, key, tkey in ((0, "r_min", "theta_min"), (k - 1, "r_max", "theta_max")):
        y = Y[:, col]
        x = V @ y
        dense = np.linalg.norm(Ht @ x - th[col] * x)
        assert abs(r[tkey] - th[col]) < 1e-12
        assert abs(r[key] - dense) <= 1e-9 * max(dense, 1e-3), (name, key, r[key], dense)
        assert abs(be[k - 1] * abs(y[0]) - dense) > 1e-6, (name, key)
