"""Pins for the oracle's MINRES (App. A, Alg. 2)."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import minres, model, precond
from workloads import disorder_fields, gaussian_vector


def test_two_eigenvalue_system_converges_in_two_steps():
    """A diagonal with M = |A|: the preconditioned operator has eigenvalues +1
    and -1 only, so the Krylov space has dimension 2 and MINRES is exact after
    two iterations."""
    rng = np.random.default_rng(0)
    a = rng.uniform(0.5, 3.0, 40) * rng.choice([-1.0, 1.0], 40)
    b = rng.standard_normal(40)
    x, k, hist = minres.minres(lambda v: a * v, np.zeros(40), b, 1.0 / np.abs(a), 50, 1e-13)
    assert k == 2
    assert np.allclose(x, b / a, rtol=1e-13, atol=1e-13)


def test_matches_library_minres_on_random_indefinite():
    rng = np.random.default_rng(1)
    n = 60
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    A = Q @ np.diag(np.linspace(-3, 5, n) + 0.05) @ Q.T
    A = 0.5 * (A + A.T)
    b = rng.standard_normal(n)
    mdiag = np.abs(np.diag(A)) + 1.0
    x, k, _ = minres.minres(lambda v: A @ v, np.zeros(n), b, 1.0 / mdiag, 10 * n, 1e-13)
    xl, info = spla.minres(A, b, M=np.diag(1.0 / mdiag), rtol=1e-14, maxiter=10 * n)
    xd = np.linalg.solve(A, b)
    assert np.linalg.norm(x - xd) / np.linalg.norm(xd) < 1e-10
    assert np.linalg.norm(x - xl) / np.linalg.norm(xd) < 1e-8


@pytest.mark.parametrize("L,h,kind", [(10, 3.0, "row"), (12, 2.0, "row"), (10, 3.0, "jacobi"), (10, 3.0, "id")])
def test_heisenberg_solve_matches_dense(L, h, kind):
    H = model.hamiltonian_csr(L, disorder_fields(L, h, 0))
    Hd = H.toarray()
    w = np.linalg.eigvalsh(Hd)
    sigma = 0.5 * (w[0] + w[-1])
    b = gaussian_vector(H.shape[0], 7)
    b /= np.linalg.norm(b)
    A = precond.shifted(H, sigma)
    m = precond.preconditioner_diagonal(H, sigma, kind)
    x, k, hist = minres.minres(lambda v: A @ v, np.zeros_like(b), b, 1.0 / m, 200000, 1e-12)
    xd = minres.solve_dense(Hd, sigma, b)
    assert np.linalg.norm(x - xd) / np.linalg.norm(xd) < 1e-8
    # |phi_k| never increases (minimum-residual property)
    assert np.all(np.diff(hist) <= 1e-14 * hist[0])
    # |phi_k| is the M^{-1}-norm of the true residual
    r = b - A @ x
    assert abs(np.sqrt(r @ (r / m)) - hist[-1]) < 1e-10
    assert hist[-1] < 1e-12


def test_row_norm_beats_identity_in_iterations():
    """Sec. IV A: the row-norm preconditioner reduces the work (fewer iterations)."""
    L = 12
    H = model.hamiltonian_csr(L, disorder_fields(L, 3.0, 0))
    w = np.linalg.eigvalsh(H.toarray())
    sigma = 0.5 * (w[0] + w[-1])
    b = gaussian_vector(H.shape[0], 7)
    b /= np.linalg.norm(b)
    A = precond.shifted(H, sigma)
    its = {}
    for kind in ("row", "id"):
        m = precond.preconditioner_diagonal(H, sigma, kind)
        its[kind] = minres.minres(lambda v: A @ v, np.zeros_like(b), b, 1.0 / m, 100000, 1e-10)[1]
    assert its["row"] < its["id"]
