"""Independent references used to pin the oracle (test-only).

Nothing here calls the oracle's C code: dense Hamiltonians are assembled from
Kronecker products of ring adjacency matrices or straight from the hopping
formula, spectra come from numpy.linalg.eigh, and random start vectors come
from numpy's own Philox4x64-10.
"""
import math

import numpy as np


def ring(L: int) -> np.ndarray:
    """Adjacency of a periodic ring as a sum over the two neighbour slots (L=1, 2 keep both)."""
    A = np.zeros((L, L))
    for x in range(L):
        A[x, (x - 1) % L] += 1.0
        A[x, (x + 1) % L] += 1.0
    return A


def clean_lattice_dense(L, t=1.0):
    """-t times the adjacency of a periodic lattice with extents L (1, 2 or 3 axes),
    site index x + Lx (y + Ly z): kron ordering has the slowest axis first."""
    L = list(L)
    H = None
    n = int(np.prod(L))
    for ax in range(len(L)):
        mats = [np.eye(Lc) for Lc in L]
        mats[ax] = ring(L[ax])
        K = np.array([[1.0]])
        for m in reversed(mats):          # slowest axis (last) first in kron
            K = np.kron(K, m)
        H = K if H is None else H + K
    return -t * H if n else H


def spin_lattice_dense(L, theta, phi, t=1.0):
    """H_ij = -t [cos(th_i/2) cos(th_j/2) + sin(th_i/2) sin(th_j/2) e^{-i(phi_i - phi_j)}]
    summed over the periodic neighbour slots, written from the hopping formula."""
    dims = len(L)
    L = list(L) + [1] * (3 - len(L))
    Lx, Ly, Lz = L
    N = Lx * Ly * Lz
    H = np.zeros((N, N), dtype=complex)
    for z in range(Lz):
        for y in range(Ly):
            for x in range(Lx):
                i = x + Lx * (y + Ly * z)
                for ax in range(dims):
                    for d in (-1, 1):
                        c = [x, y, z]
                        c[ax] = (c[ax] + d) % L[ax]
                        j = c[0] + Lx * (c[1] + Ly * c[2])
                        tij = (math.cos(theta[i] / 2) * math.cos(theta[j] / 2)
                               + math.sin(theta[i] / 2) * math.sin(theta[j] / 2)
                               * np.exp(-1j * (phi[i] - phi[j])))
                        H[i, j] += -t * tij
    return H


def csr_dense(csr):
    H = np.zeros((csr.n, csr.n), dtype=complex)
    for i in range(csr.n):
        for k in range(csr.row_ptr[i], csr.row_ptr[i + 1]):
            H[i, csr.col[k]] += csr.val_re[k] + (1j * csr.val_im[k] if csr.val_im is not None else 0)
    return H


def cheb_T(n, x):
    """T_n(x) = cos(n arccos x) (Sec. II-A definition), for |x| <= 1."""
    return np.cos(n * np.arccos(np.clip(x, -1.0, 1.0)))


def numpy_philox_block(counter, key):
    """Philox4x64-10 block at `counter` from numpy's implementation (which increments the
    256-bit counter before producing a block, so start it one below)."""
    c = int(counter[0]) + (int(counter[1]) << 64) + (int(counter[2]) << 128) + (int(counter[3]) << 192)
    c = (c - 1) % (1 << 256)
    words = [(c >> (64 * w)) & ((1 << 64) - 1) for w in range(4)]
    bg = np.random.Philox(counter=np.array(words, dtype=np.uint64),
                          key=np.array([int(key[0]), int(key[1])], dtype=np.uint64))
    return bg.random_raw(4)


def phase_factors(bits=30):
    """w_j = exp(2 pi i 2^j / 2^bits) by the half-angle recurrence from exp(i pi) and exp(i pi/2)."""
    w = [None] * bits
    c, s = -1.0, 0.0
    w[bits - 1] = (c, s)
    c, s = 0.0, 1.0
    w[bits - 2] = (c, s)
    for m in range(3, bits + 1):
        ch = math.sqrt((1.0 + c) / 2.0)
        s = s / (2.0 * ch)
        c = ch
        w[bits - m] = (c, s)
    return w


_W = phase_factors()


def phase_of_word(w):
    """exp(2 pi i k / 2^30), k = top 30 bits of w, as the ordered product of w_j over set bits."""
    k = w >> 34
    z = None
    for j in range(30):
        if (k >> j) & 1:
            if z is None:
                z = _W[j]
            else:
                zr, zi = z
                wr, wi = _W[j]
                z = (zr * wr - zi * wi, zr * wi + zi * wr)
    return complex(*(z or (1.0, 0.0)))


def start_vectors_numpy(kind, seed, instance, N, R):
    """The start vectors of the method drawn with numpy's Philox: counter (i, r//4, instance, 0),
    key (seed, 4), word r % 4; Rademacher from the top bit, phase from the top 30 bits."""
    X = np.zeros((R, N), dtype=complex)
    for r in range(R):
        for i in range(N):
            if kind == 2:
                X[r, i] = 1.0 if i == (instance + r) % N else 0.0
                continue
            w = int(numpy_philox_block([i, r // 4, instance, 0], [seed, 4])[r % 4])
            if kind == 0:
                X[r, i] = -1.0 if (w >> 63) else 1.0
            else:
                X[r, i] = phase_of_word(w)
    return X


def estimator_from_eigh(Ht, X, M):
    """(1/(N R)) sum_r <xi_r| T_n(H~) |xi_r> = (1/(N R)) sum_r sum_k |<psi_k|xi_r>|^2 T_n(E~_k)."""
    E, V = np.linalg.eigh(Ht)
    R, N = X.shape
    w = (np.abs(V.conj().T @ X.T) ** 2).sum(axis=1)          # sum_r |<psi_k|xi_r>|^2
    return np.array([np.dot(w, cheb_T(n, E)) for n in range(M)]) / (N * R)


def exact_moments_from_eigh(Ht, M):
    E = np.linalg.eigvalsh(Ht)
    return np.array([cheb_T(n, E).mean() for n in range(M)])
