"""Seeded synthetic inputs for the KPM workloads.

This module only draws model inputs (disorder, spin textures, lattice sizes,
request streams).  It holds none of the method's arithmetic: no rescaling, no
recursion, no moments.  Both the HIP path and the CPU oracle take what it
returns as plain arrays, so neither depends on the other.

Random streams: numpy's Philox4x64-10 with key (master seed, tag), one tag per
kind of input.  The vectors the method itself draws use tag 4 and are drawn
by the method (on the device, and independently in the oracle), not here.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np

TAG_DISORDER, TAG_SPINS, TAG_REDRAW, TAG_VECTORS, TAG_SIZE, TAG_ARRIVAL, TAG_REQUEST, TAG_DENSE = 1, 2, 3, 4, 5, 6, 7, 8

HOP_REAL, HOP_SPIN = 0, 1
VEC_RADEMACHER, VEC_PHASE, VEC_UNIT = 0, 1, 2


def rng(seed: int, tag: int) -> np.random.Generator:
    return np.random.Generator(np.random.Philox(key=[int(seed) & (2**64 - 1), int(tag)]))


@dataclass
class Lattice:
    """A periodic square (dim 2) or cubic (dim 3) tight-binding lattice.

    Site index i = x + Lx (y + Ly z).  hop == HOP_REAL: H_ij = -t on every
    nearest-neighbour bond.  hop == HOP_SPIN: H_ij = -t u_i^dag u_j with the
    spinor u_i = (cos(theta_i/2), e^{i phi_i} sin(theta_i/2)), passed as the
    (N, 3) array (cos(theta/2), sin(theta/2) cos(phi), sin(theta/2) sin(phi)).
    onsite: the diagonal H_ii (None means zero).
    """
    dim: int
    L: Tuple[int, int, int]
    t: float = 1.0
    hop: int = HOP_REAL
    onsite: Optional[np.ndarray] = None
    spinor: Optional[np.ndarray] = None
    theta: Optional[np.ndarray] = None
    phi: Optional[np.ndarray] = None

    @property
    def N(self) -> int:
        return int(self.L[0] * self.L[1] * (self.L[2] if self.dim == 3 else 1))


@dataclass
class CSR:
    """A general sparse Hermitian matrix in compressed-row form."""
    n: int
    row_ptr: np.ndarray
    col: np.ndarray
    val_re: np.ndarray
    val_im: Optional[np.ndarray] = None


def anderson_onsite(N: int, W: float, seed: int) -> np.ndarray:
    """On-site energies uniform in [-W/2, W/2]."""
    return rng(seed, TAG_DISORDER).uniform(-W / 2.0, W / 2.0, size=N)


def spins_uniform(N: int, seed: int, tag: int = TAG_SPINS):
    """Classical spins uniform on the sphere: cos(theta) = 1 - 2 u1, phi = 2 pi u2."""
    g = rng(seed, tag)
    u = g.random(size=(2, N))
    theta = np.arccos(1.0 - 2.0 * u[0])
    phi = 2.0 * np.pi * u[1]
    return theta, phi


def spinor_of(theta: np.ndarray, phi: np.ndarray) -> np.ndarray:
    """(cos(theta/2), sin(theta/2) cos(phi), sin(theta/2) sin(phi)) per site, shape (N, 3)."""
    c = np.cos(theta / 2.0)
    s = np.sin(theta / 2.0)
    return np.ascontiguousarray(np.stack([c, s * np.cos(phi), s * np.sin(phi)], axis=1))


def square_lattice(L: int, t: float = 1.0, W: float = 0.0, seed: int = 0) -> Lattice:
    onsite = anderson_onsite(L * L, W, seed) if W > 0 else None
    return Lattice(dim=2, L=(L, L, 1), t=t, hop=HOP_REAL, onsite=onsite)


def cubic_lattice(L: int, t: float = 1.0, W: float = 0.0, seed: int = 0) -> Lattice:
    onsite = anderson_onsite(L ** 3, W, seed) if W > 0 else None
    return Lattice(dim=3, L=(L, L, L), t=t, hop=HOP_REAL, onsite=onsite)


def spin_cubic_lattice(L: int, t: float = 1.0, seed: int = 0, theta=None, phi=None) -> Lattice:
    N = L ** 3
    if theta is None:
        theta, phi = spins_uniform(N, seed)
    return Lattice(dim=3, L=(L, L, L), t=t, hop=HOP_SPIN, spinor=spinor_of(theta, phi),
                   theta=theta, phi=phi)


def lattice_to_csr(lat: Lattice) -> CSR:
    """The same Hamiltonian H (unscaled) in CSR form.  Each row stores the diagonal first,
    then the neighbour slots in the order -x, +x, -y, +y[, -z, +z]; a slot that wraps onto an
    already-listed column is kept as a separate entry (entries are summed)."""
    N = lat.N
    Lx, Ly = lat.L[0], lat.L[1]
    Lz = lat.L[2] if lat.dim == 3 else 1
    i = np.arange(N)
    x, y, z = i % Lx, (i // Lx) % Ly, i // (Lx * Ly)
    cols = [i]
    vre = [lat.onsite if lat.onsite is not None else np.zeros(N)]
    vim = [np.zeros(N)]
    axes = [(x, Lx), (y, Ly)] + ([(z, Lz)] if lat.dim == 3 else [])
    for ax, (c, Lc) in enumerate(axes):
        for d in (-1, +1):
            cn = (c + d) % Lc
            coords = [x, y, z]
            coords[ax] = cn
            j = coords[0] + Lx * (coords[1] + Ly * coords[2])
            cols.append(j)
            if lat.hop == HOP_REAL:
                vre.append(np.full(N, -lat.t))
                vim.append(np.zeros(N))
            else:
                # H_ij = -t u_i^dag u_j written out from theta and phi
                th, ph = lat.theta, lat.phi
                tij = (np.cos(th[i] / 2) * np.cos(th[j] / 2)
                       + np.sin(th[i] / 2) * np.sin(th[j] / 2) * np.exp(-1j * (ph[i] - ph[j])))
                vre.append(-lat.t * tij.real)
                vim.append(-lat.t * tij.imag)
    ns = len(cols)
    col = np.stack(cols, axis=1).reshape(-1).astype(np.int32)
    val_re = np.stack(vre, axis=1).reshape(-1)
    val_im = np.stack(vim, axis=1).reshape(-1)
    row_ptr = np.arange(N + 1, dtype=np.int64) * ns
    return CSR(n=N, row_ptr=row_ptr, col=col, val_re=val_re,
               val_im=None if lat.hop == HOP_REAL else val_im)


def random_hermitian_csr(n: int, nnz_per_row: int, seed: int, complex_values: bool = True,
                         diag_scale: float = 1.0) -> CSR:
    """A random sparse Hermitian matrix with unsorted, duplicate-free off-diagonal columns and
    the diagonal stored at a random position inside each row."""
    g = rng(seed, TAG_REQUEST)
    pairs = set()
    for i in range(n):
        k = 0
        while k < nnz_per_row // 2:
            j = int(g.integers(0, n))
            if j != i and (i, j) not in pairs:
                pairs.add((i, j))
                pairs.add((j, i))
                k += 1
    rows = [[] for _ in range(n)]
    vals = {}
    for (i, j) in sorted(pairs):
        if i < j:
            v = g.normal() + (1j * g.normal() if complex_values else 0.0)
            vals[(i, j)] = v
            vals[(j, i)] = np.conj(v)
    for (i, j) in pairs:
        rows[i].append(j)
    row_ptr = [0]
    col, vre, vim = [], [], []
    for i in range(n):
        js = list(rows[i])
        g.shuffle(js)
        pos = int(g.integers(0, len(js) + 1))
        js.insert(pos, i)
        for j in js:
            col.append(j)
            v = diag_scale * g.normal() if j == i else vals[(i, j)]
            vre.append(float(np.real(v)))
            vim.append(float(np.imag(v)))
        row_ptr.append(len(col))
    return CSR(n=n, row_ptr=np.array(row_ptr, dtype=np.int64), col=np.array(col, dtype=np.int32),
               val_re=np.array(vre), val_im=np.array(vim) if complex_values else None)


# ----------------------------------------------------------------------------
# the five workloads
# ----------------------------------------------------------------------------
def config1() -> dict:
    """2D square 32x32, periodic, t=1, on-site uniform[-0.5, 0.5]; FP64, M=256, R=8 +-1 vectors,
    Jackson DoS on 1024 Chebyshev points."""
    seed = 1001
    return dict(lattice=square_lattice(32, t=1.0, W=1.0, seed=seed), M=256, R=8,
                vec=VEC_RADEMACHER, seed=seed, K=1024, name="square2d_L32_M256_R8")


def config2() -> dict:
    """3D cubic 64^3, periodic, spin hopping from spins uniform on the sphere; M=1024,
    R=32 random-phase vectors."""
    seed = 1002
    return dict(lattice=spin_cubic_lattice(64, t=1.0, seed=seed), M=1024, R=32,
                vec=VEC_PHASE, seed=seed, name="spin_cubic_L64_M1024_R32")


def config3(count: int = 256, Lmin: int = 16, Lmax: int = 48) -> dict:
    """count 3D spin-hopping cubes, L uniform in {Lmin..Lmax}; each is the base texture (one
    spin per coordinate of a Lmax^3 cube, restricted to L^3) with 1..8 spins re-drawn."""
    seed = 1003
    Ls = rng(seed, TAG_SIZE).integers(Lmin, Lmax + 1, size=count)
    base_theta, base_phi = spins_uniform(Lmax ** 3, seed)
    base_theta = base_theta.reshape(Lmax, Lmax, Lmax)   # [z][y][x]
    base_phi = base_phi.reshape(Lmax, Lmax, Lmax)
    lats = []
    g = rng(seed, TAG_REDRAW)
    for h, L in enumerate(Ls):
        L = int(L)
        th = np.ascontiguousarray(base_theta[:L, :L, :L]).reshape(-1).copy()
        ph = np.ascontiguousarray(base_phi[:L, :L, :L]).reshape(-1).copy()
        k = int(g.integers(1, 9))
        sites = g.choice(L ** 3, size=k, replace=False)
        u = g.random(size=(2, k))
        th[sites] = np.arccos(1.0 - 2.0 * u[0])
        ph[sites] = 2.0 * np.pi * u[1]
        lats.append(spin_cubic_lattice(L, t=1.0, theta=th, phi=ph))
    return dict(lattices=lats, M=512, R=16, vec=VEC_PHASE, seed=seed,
                name=f"batched_spin_cubic_{count}x_L{Lmin}-{Lmax}_M512_R16")


def csr_to_dense(c: CSR) -> np.ndarray:
    """The real part of a CSR matrix as a dense row-major float64 array (entries with equal
    (row, col) summed)."""
    H = np.zeros((c.n, c.n))
    rows = np.repeat(np.arange(c.n), np.diff(c.row_ptr))
    np.add.at(H, (rows, c.col), c.val_re)
    return H


def dense_symmetric(D: int, seed: int) -> np.ndarray:
    """A dense real symmetric D x D matrix with independent N(0, 1/(2D)) entries above the diagonal
    and N(0, 1/D) on it (the Gaussian orthogonal ensemble, spectrum ~ [-2, 2]), row-major float64."""
    g = rng(seed, TAG_DENSE)
    X = g.normal(size=(D, D)) / np.sqrt(2.0 * D)
    return np.ascontiguousarray(X + X.T)


def dense_workloads() -> dict:
    """The shapes of the paper's dense-H experiments (Sec. IV): R x S = 1792 vectors (+-1).
    E1: the 10x10x10 cubic lattice with zero diagonal and -1 hopping as a dense matrix (D = 1000),
    M = 1024; E3: D = 128, M = 2048; E4: D = 4096 (the largest H_SIZE), M = 128.  E3 and E4 use
    dense_symmetric matrices (the paper does not specify its matrices)."""
    seed = 1006
    return dict(R=1792, vec=VEC_RADEMACHER, seed=seed,
                shapes={"E1_lattice_D1000_M1024": ("lattice", 1000, 1024),
                        "E3_D128_M2048": ("random", 128, 2048),
                        "E4_D4096_M128": ("random", 4096, 128)})


def config4() -> dict:
    """2D square 2048x2048, Anderson disorder uniform[-1, 1], FP32 vectors, M=4096, R=64."""
    seed = 1004
    return dict(lattice=square_lattice(2048, t=1.0, W=2.0, seed=seed), M=4096, R=64,
                vec=VEC_RADEMACHER, seed=seed, name="anderson2d_L2048_M4096_R64")


@dataclass
class Request:
    rid: int
    arrival: float
    lattice: Lattice
    M: int
    R: int
    vec: int
    seed: int


def config5_stream(n_requests: int, rate: float, seed: int = 1005, logN_min: float = 12.0,
                   logN_max: float = 24.0, Ms=(256, 1024, 4096, 8192), Rmin: int = 8,
                   Rmax: int = 64) -> List[Request]:
    """Poisson arrivals (rate per second); N log-uniform on [2^logN_min, 2^logN_max]; d in {2,3};
    L = round(N^(1/d)); real (Anderson W in {1,2}) or spin hopping; M from Ms; R in [Rmin, Rmax]."""
    ga = rng(seed, TAG_ARRIVAL)
    gr = rng(seed, TAG_REQUEST)
    t = 0.0
    out = []
    for rid in range(n_requests):
        t += float(ga.exponential(1.0 / rate))
        logN = float(gr.uniform(logN_min, logN_max))
        d = 2 if gr.random() < 0.5 else 3
        L = max(3, int(round(2.0 ** (logN / d))))
        spin = gr.random() < 0.5
        M = int(Ms[int(gr.integers(0, len(Ms)))])
        R = int(gr.integers(Rmin, Rmax + 1))
        rseed = int(gr.integers(0, 2**62))
        if spin:
            N = L ** d
            th, ph = spins_uniform(N, rseed)
            lat = Lattice(dim=d, L=(L, L, L if d == 3 else 1), t=1.0, hop=HOP_SPIN,
                          spinor=spinor_of(th, ph), theta=th, phi=ph)
        else:
            W = 1.0 if gr.random() < 0.5 else 2.0
            lat = square_lattice(L, W=W, seed=rseed) if d == 2 else cubic_lattice(L, W=W, seed=rseed)
        out.append(Request(rid=rid, arrival=t, lattice=lat, M=M, R=R, vec=VEC_PHASE if spin else VEC_RADEMACHER,
                           seed=rseed))
    return out
