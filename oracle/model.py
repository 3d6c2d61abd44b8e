"""Eq. (1) of the paper in the S^z basis of the S^z = 0 sector (Sec. I).

H = sum_{j=1}^{L} ( S_j . S_{j+1} - h_j S^z_j ),  S_{L+1} = S_1,  J = 1.

Site j is bit j-1 of the state integer; bit value 1 means S^z_j = +1/2.
The sector basis is every L-bit integer with L/2 set bits, ascending
(dimension C(L, L/2), Sec. III). In that basis H is real symmetric:

* diagonal: sum over bonds of s_j s_{j+1} (+1/4 parallel, -1/4 antiparallel)
  minus sum_j h_j s_j, with s_j = bit_{j-1} - 1/2;
* off-diagonal: (S^+_j S^-_{j+1} + S^-_j S^+_{j+1}) / 2 swaps an antiparallel
  pair on bond j with amplitude 1/2.

``hamiltonian_kron`` builds H on the full 2^L space from 2x2 spin matrices and
Kronecker products; it shares nothing with the bit-manipulation build and is
used to pin it.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def popcount(a: np.ndarray, L: int) -> np.ndarray:
    a = np.asarray(a, dtype=np.int64)
    c = np.zeros(a.shape, dtype=np.int64)
    for b in range(L):
        c += (a >> b) & 1
    return c


def sector_states(L: int) -> np.ndarray:
    """All L-bit integers with L/2 set bits, ascending (the S^z = 0 sector)."""
    if L < 2 or L % 2:
        raise ValueError("L must be even and >= 2")
    allst = np.arange(1 << L, dtype=np.int64)
    return allst[popcount(allst, L) == L // 2]


def spin(states: np.ndarray, j: int) -> np.ndarray:
    """s_j(alpha) = S^z eigenvalue of site j (1-based) in each state."""
    return ((states >> (j - 1)) & 1).astype(np.float64) - 0.5


def bonds(L: int):
    """Bond j (1-based) joins sites j and j+1, with site L+1 = site 1."""
    return [(j, j % L + 1) for j in range(1, L + 1)]


def diagonal(L: int, h: np.ndarray, states: np.ndarray) -> np.ndarray:
    """<alpha|H|alpha> = sum_j s_j s_{j+1} - sum_j h_j s_j."""
    h = np.asarray(h, dtype=np.float64)
    d = np.zeros(states.shape[0], dtype=np.float64)
    for (a, b) in bonds(L):
        d += spin(states, a) * spin(states, b)
    for j in range(1, L + 1):
        d -= h[j - 1] * spin(states, j)
    return d


def offdiagonal_triplets(L: int, states: np.ndarray):
    """(row, col, value) of every nonzero off-diagonal element <beta|H|alpha>.

    For each bond with antiparallel spins in alpha, beta = alpha with the two
    spins swapped and the element is 1/2. Row indices come from a sorted
    lookup of beta in the ascending basis.
    """
    rows, cols = [], []
    idx = np.arange(states.shape[0], dtype=np.int64)
    for (a, b) in bonds(L):
        ba = (states >> (a - 1)) & 1
        bb = (states >> (b - 1)) & 1
        anti = ba != bb
        flipped = states[anti] ^ ((1 << (a - 1)) | (1 << (b - 1)))
        r = np.searchsorted(states, flipped)
        assert np.array_equal(states[r], flipped)
        rows.append(r)
        cols.append(idx[anti])
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    return rows, cols, np.full(rows.shape[0], 0.5)


def hamiltonian_csr(L: int, h: np.ndarray) -> sp.csr_matrix:
    """H of Eq. (1) restricted to the S^z = 0 sector, as a CSR matrix."""
    states = sector_states(L)
    n = states.shape[0]
    r, c, v = offdiagonal_triplets(L, states)
    off = sp.coo_matrix((v, (r, c)), shape=(n, n))
    return (off + sp.diags(diagonal(L, h, states))).tocsr()


def hamiltonian_dense(L: int, h: np.ndarray) -> np.ndarray:
    return hamiltonian_csr(L, h).toarray()


def hamiltonian_xy_csr(L: int) -> sp.csr_matrix:
    """Only the spin-flip part (1/2) sum_j (S^+_j S^-_{j+1} + h.c.)."""
    states = sector_states(L)
    n = states.shape[0]
    r, c, v = offdiagonal_triplets(L, states)
    return sp.coo_matrix((v, (r, c)), shape=(n, n)).tocsr()


# ---------------------------------------------------------------------------
# Independent construction on the full 2^L space (pin for the sector build).

_SZ = np.array([[-0.5, 0.0], [0.0, 0.5]], dtype=np.complex128)   # basis (bit 0, bit 1)
_SP = np.array([[0.0, 0.0], [1.0, 0.0]], dtype=np.complex128)    # raises bit 0 -> bit 1
_SM = _SP.T.copy()
_SX = 0.5 * (_SP + _SM)
_SY = (_SP - _SM) / 2j


def _site_op(op: np.ndarray, j: int, L: int) -> np.ndarray:
    """op acting on site j (bit j-1); the last Kronecker factor is bit 0."""
    k = j - 1
    return np.kron(np.kron(np.eye(1 << (L - 1 - k)), op), np.eye(1 << k))


def hamiltonian_kron(L: int, h: np.ndarray) -> np.ndarray:
    """Eq. (1) on the full 2^L space from spin matrices (complex dtype)."""
    dim = 1 << L
    H = np.zeros((dim, dim), dtype=np.complex128)
    ops = {}
    for j in range(1, L + 1):
        ops[j] = tuple(_site_op(o, j, L) for o in (_SX, _SY, _SZ))
    for (a, b) in bonds(L):
        for t in range(3):
            H += ops[a][t] @ ops[b][t]
    for j in range(1, L + 1):
        H -= h[j - 1] * ops[j][2]
    return H


def total_sz_kron(L: int) -> np.ndarray:
    return sum(_site_op(_SZ, j, L) for j in range(1, L + 1))
