"""Pins for the oracle's Hamiltonian (Eq. (1)) and basis (Sec. I, III)."""
import json
import math
import os

import numpy as np
import pytest

from oracle import model, precond
from workloads import disorder_fields

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")))


@pytest.mark.parametrize("L", [4, 6, 8, 10, 12, 14])
def test_basis_dimension_and_order(L):
    st = model.sector_states(L)
    assert st.shape[0] == math.comb(L, L // 2)
    assert np.all(np.diff(st) > 0)
    assert np.all(model.popcount(st, L) == L // 2)
    # brute force with Python integers
    brute = [s for s in range(1 << L) if bin(s).count("1") == L // 2]
    assert st.tolist() == brute


@pytest.mark.parametrize("L,seed", [(4, 0), (6, 1), (8, 2)])
def test_sector_build_equals_kronecker_projection(L, seed):
    h = disorder_fields(L, 3.0, seed)
    Hk = model.hamiltonian_kron(L, h)
    assert np.abs(Hk.imag).max() == 0.0
    # S^z conservation: H commutes with total S^z on the full space
    Sz = model.total_sz_kron(L)
    assert np.abs(Hk @ Sz - Sz @ Hk).max() < 1e-13
    st = model.sector_states(L)
    Hp = Hk.real[np.ix_(st, st)]
    Hs = model.hamiltonian_dense(L, h)
    assert np.abs(Hp - Hs).max() < 1e-14
    # nothing couples the sector to the rest of the space
    rest = np.setdiff1d(np.arange(1 << L), st)
    assert np.abs(Hk.real[np.ix_(rest, st)]).max() == 0.0


def test_ring4_spectrum_closed_form():
    w = np.linalg.eigvalsh(model.hamiltonian_dense(4, np.zeros(4)))
    assert np.allclose(w, GOLD["ring4_spectrum_h0"]["value"], atol=1e-13)


def test_ring6_ground_energy_closed_form():
    w = np.linalg.eigvalsh(model.hamiltonian_dense(6, np.zeros(6)))
    assert abs(w[0] - (-1 - math.sqrt(13) / 2)) < 1e-12
    assert abs(w[0] - GOLD["ring6_ground_energy_h0"]["value"]) < 1e-12


@pytest.mark.parametrize("L", [4, 6, 8, 10, 12])
def test_trace_closed_form(L):
    h = disorder_fields(L, 4.0, L)
    H = model.hamiltonian_csr(L, h)
    tr = H.diagonal().sum()
    assert abs(tr - (-math.comb(L - 2, L // 2 - 1))) < 1e-10
    assert abs(tr - (L // 2) * (math.comb(L - 2, L // 2) - math.comb(L - 2, L // 2 - 1))) < 1e-10


@pytest.mark.parametrize("L", [8, 10])
def test_spectrum_invariances(L):
    h = disorder_fields(L, 3.0, 5)
    w = np.linalg.eigvalsh(model.hamiltonian_dense(L, h))
    for hh in (np.roll(h, 1), h[::-1], -h):
        w2 = np.linalg.eigvalsh(model.hamiltonian_dense(L, hh))
        assert np.abs(w - w2).max() < 1e-12
    # a uniform field shift does nothing in S^z_tot = 0
    w3 = np.linalg.eigvalsh(model.hamiltonian_dense(L, h + 0.7))
    assert np.abs(w - w3).max() < 1e-12


def test_symmetric():
    H = model.hamiltonian_csr(12, disorder_fields(12, 2.0, 0))
    assert abs(H - H.T).max() == 0.0


@pytest.mark.parametrize("L,seed", [(6, 0), (8, 3)])
def test_row_norm_matches_kronecker_rows(L, seed):
    """r_i^2 = (a_ii - sigma)^2 + (number of antiparallel bonds)/4, with the
    off-diagonal count taken from the independent Kronecker build."""
    h = disorder_fields(L, 3.0, seed)
    sigma = 0.37
    st = model.sector_states(L)
    Hp = model.hamiltonian_kron(L, h).real[np.ix_(st, st)]
    off = Hp - np.diag(np.diag(Hp))
    nnz = (off != 0).sum(axis=1)
    assert np.all(off[off != 0] == 0.5)
    r = precond.row_norm_diagonal(model.hamiltonian_csr(L, h), sigma)
    assert np.allclose(r ** 2, (np.diag(Hp) - sigma) ** 2 + nnz / 4.0, rtol=0, atol=1e-13)
    assert r.min() >= 1 / math.sqrt(2) - 1e-15


@pytest.mark.parametrize("L,seed,sigma", [(6, 1, 0.37), (8, 4, -0.61)])
def test_jacobi_diagonal_matches_kronecker_diagonal(L, seed, sigma):
    """Jacobi preconditioner of Sec. II: m_i = |a_ii - sigma| with a_ii read
    off the independent Kronecker build projected on the sector (a wrong sign
    of the shift, a dropped field term or a row permutation fails here; MINRES
    itself converges for any SPD M, so the solve tests cannot see it)."""
    h = disorder_fields(L, 3.0, seed)
    st = model.sector_states(L)
    a = np.diag(model.hamiltonian_kron(L, h).real[np.ix_(st, st)])
    m = precond.jacobi_diagonal(model.hamiltonian_csr(L, h), sigma)
    assert np.allclose(m, np.abs(a - sigma), rtol=0, atol=1e-13)
    # the same definition through the dispatcher, and on a dense matrix
    assert np.array_equal(precond.preconditioner_diagonal(model.hamiltonian_csr(L, h), sigma,
                                                          "jacobi"), m)
    assert np.allclose(precond.jacobi_diagonal(model.hamiltonian_dense(L, h), sigma), m,
                       rtol=0, atol=0)
    # h = 0 on a ring: a_ii = (L - 2 N_anti) / 4 exactly (N_anti antiparallel bonds)
    z = model.hamiltonian_csr(L, np.zeros(L))
    nanti = np.array([bin(s ^ (((s << 1) | (s >> (L - 1))) & ((1 << L) - 1))).count("1")
                      for s in st])
    assert np.array_equal(precond.jacobi_diagonal(z, 0.0), np.abs((L - 2 * nanti) / 4.0))
