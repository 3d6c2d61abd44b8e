"""Pins for the oracle's shift-invert Lanczos (Alg. 1) and eigenpair selection."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import lanczos, minres, model, precond
from workloads import disorder_fields, start_vector


def _setup(L, h, seed):
    H = model.hamiltonian_csr(L, disorder_fields(L, h, seed))
    Hd = H.toarray()
    w = np.linalg.eigvalsh(Hd)
    return H, Hd, w, 0.5 * (w[0] + w[-1])


@pytest.mark.parametrize("L,h,nev", [(10, 3.0, 6), (12, 3.0, 10)])
def test_si_lanczos_exact_solves_matches_dense(L, h, nev):
    H, Hd, w, sigma = _setup(L, h, 0)
    A = Hd - sigma * np.eye(Hd.shape[0])
    lu = np.linalg.inv(A)
    out = lanczos.si_lanczos(lambda v: lu @ v, start_vector(Hd.shape[0], 0), 400, sigma,
                             nev=nev, hnorm=max(abs(w[0]), abs(w[-1])), eig_tol=1e-12)
    E_ref, V_ref = lanczos.eigenpairs_dense(Hd, sigma, nev)
    assert np.allclose(out["evals"], E_ref, rtol=0, atol=1e-10)
    ov = np.abs(np.sum(out["evecs"] * V_ref, axis=0))
    assert np.all(1 - ov < 1e-9)
    res = lanczos.eigen_residuals(Hd, out["evals"], out["evecs"])
    assert res.max() < 1e-9


def test_si_lanczos_with_minres_inner_solves():
    L, h, nev = 10, 3.0, 4
    H, Hd, w, sigma = _setup(L, h, 1)
    A = precond.shifted(H, sigma)
    m = precond.row_norm_diagonal(H, sigma)
    solve = lambda v: minres.minres(lambda u: A @ u, np.zeros_like(v), v, 1.0 / m, 100000, 1e-13)[0]  # noqa
    out = lanczos.si_lanczos(solve, start_vector(Hd.shape[0], 3), 200, sigma, nev=nev,
                             hnorm=max(abs(w[0]), abs(w[-1])), eig_tol=1e-12)
    E_ref, _ = lanczos.eigenpairs_dense(Hd, sigma, nev)
    assert np.allclose(out["evals"], E_ref, rtol=0, atol=1e-10)


def test_breakdown_on_eigenvector_start():
    """Starting from an eigenvector, beta_2 = 0 (up to rounding) and the single
    Ritz value is sigma + 1/theta = the eigenvalue."""
    H, Hd, w, sigma = _setup(8, 2.0, 2)
    _, V = np.linalg.eigh(Hd)
    lu = np.linalg.inv(Hd - sigma * np.eye(Hd.shape[0]))
    out = lanczos.si_lanczos(lambda v: lu @ v, V[:, 11], 1, sigma, nev=1)
    assert out["steps"] == 1
    assert abs(out["beta"][0]) < 1e-10
    assert abs(out["evals"][0] - w[11]) < 1e-12


def test_selection_rule():
    ev = np.array([-1.0, 0.0, 0.5, 1.0, 2.0])
    idx = lanczos.select_nearest(ev, 0.5, 3)
    assert ev[idx].tolist() == [0.0, 0.5, 1.0]
    idx = lanczos.select_nearest(ev, 0.25, 2)     # tie between 0.0 and 0.5 is not a tie
    assert ev[idx].tolist() == [0.0, 0.5]
    idx = lanczos.select_nearest(np.array([0.0, 1.0, 2.0]), 1.5, 1)   # tie 1.0 vs 2.0 -> lower
    assert idx.tolist() == [1]


def test_dense_selection_agrees_with_library_shift_invert():
    H, Hd, w, sigma = _setup(12, 3.0, 4)
    E1, V1 = lanczos.eigenpairs_dense(Hd, sigma, 8)
    E2, V2 = lanczos.eigenpairs_shift_invert_sparse(H, sigma, 8)
    assert np.allclose(E1, E2, atol=1e-11)
    assert np.all(1 - np.abs(np.sum(V1 * V2, axis=0)) < 1e-9)


def test_extremal_eigenvalues_sparse_vs_dense():
    H, Hd, w, sigma = _setup(14, 3.0, 0)
    lo, hi = lanczos.extremal_eigenvalues(H)
    assert abs(lo - w[0]) < 1e-10 and abs(hi - w[-1]) < 1e-10
