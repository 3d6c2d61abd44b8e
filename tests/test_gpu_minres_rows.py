"""MINRES in its row-launch form (two row launches per iteration, blocks of
iterations replayed from a captured graph), the form taken from L = 16 up,
against the oracle's Alg. 2 (App. A).

Bars, from the oracle run against itself with the matrix product perturbed at
the level of FP64 rounding (2e-16 relative): converged solves at L = 16 then
differ by 3e-12 in x and by 0.2 % in the iteration count; after a fixed
number of iterations phi differs by 2e-6 (300 iterations, L = 16) to 3e-5
(1500 iterations, L = 18). Independent of the rounding path, the MINRES
identity |phi_k| = ||b - A x_k||_{M^-1} holds to 1e-13 in the oracle.
"""
import os
import sys

import numpy as np
import pytest

from oracle import lanczos, minres, model, precond
from workloads import disorder_fields, gaussian_vector

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


def dev(torch, a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda")


def host(t):
    return t.detach().cpu().numpy()


def _problem(L, h, seed, bseed=7):
    f = disorder_fields(L, h, seed)
    H = model.hamiltonian_csr(L, f)
    lo, hi = lanczos.extremal_eigenvalues(H)
    sigma = 0.5 * (lo + hi)
    bv = gaussian_vector(H.shape[0], bseed)
    bv /= np.linalg.norm(bv)
    A = precond.shifted(H, sigma)
    m = precond.preconditioner_diagonal(H, sigma, "row")
    return f, sigma, bv, A, m


def _mnorm(r, m):
    return float(np.sqrt(r @ (r / m)))


@pytest.mark.parametrize("L,seed,kmax", [(16, 0, 300), (18, 0, 1500), (18, 1, 1500)])
def test_minres_rows_bounded_vs_oracle(gpu, torch, L, seed, kmax):
    """kmax iterations (tolerance 1e-300, so both stop at kmax): phi equals the
    preconditioned norm of the true residual of the returned x, and equals
    the oracle's phi after the same number of iterations."""
    say(f"minres row form bounded L={L} seed={seed} kmax={kmax}")
    f, sigma, bv, A, m = _problem(L, 3.0, seed)
    b = gpu.Basis(L)
    x, info = gpu.minres_solve(b, f, sigma, dev(torch, bv), tol=1e-300, kmax=kmax)
    assert info.status == gpu.WARN_NOCONV and info.iters == kmax
    xh = host(x)
    assert abs(_mnorm(bv - A @ xh, m) - info.phi) <= 1e-9 * info.phi
    _, k_ref, hist = minres.minres(lambda v: A @ v, np.zeros_like(bv), bv, 1.0 / m, kmax, 0.0)
    assert k_ref == kmax
    assert abs(info.phi - hist[-1]) <= 1e-3 * hist[-1]


@pytest.mark.parametrize("precision", ["fp64", "fp32_inner"])
def test_minres_rows_converged_vs_oracle(gpu, torch, precision):
    """A converged solve at L = 16 (tol 1e-12) equals the oracle's converged
    x; in FP64 the iteration count is the oracle's within 5 %."""
    L = 16
    say(f"minres row form converged L={L} {precision}")
    f, sigma, bv, A, m = _problem(L, 3.0, 0)
    b = gpu.Basis(L)
    x, info = gpu.minres_solve(b, f, sigma, dev(torch, bv), tol=1e-12, precision=precision)
    assert info.status == 0
    xr, k_ref, _ = minres.minres(lambda v: A @ v, np.zeros_like(bv), bv, 1.0 / m, 10**6, 1e-12)
    xh = host(x)
    assert np.linalg.norm(xh - xr) <= 1e-9 * np.linalg.norm(xr)
    assert _mnorm(bv - A @ xh, m) < 1e-10
    if precision == "fp64":
        assert abs(info.iters - k_ref) <= 0.05 * k_ref + 5


def test_minres_rows_graph_replays_match_eager(gpu, torch):
    """Solves through graph replays, with other work and synchronisations
    between them, equal solves with eager launches bit for bit."""
    L = 16
    f, sigma, bv, A, m = _problem(L, 3.0, 1)
    b = gpu.Basis(L)
    os.environ["MBL_MINRES_GRAPHS"] = "0"
    try:
        ws_e = gpu.Workspace(b, 0)
        xe0, _ = gpu.minres_solve(b, f, sigma, dev(torch, bv), tol=1e-6, kmax=100, ws=ws_e)
    finally:
        del os.environ["MBL_MINRES_GRAPHS"]
    ws_g = gpu.Workspace(b, 0)
    # the second solve replays the graph captured by the first; the third
    # changes the shift, so the graph is captured again
    for trial, (ds, tol, kmax) in enumerate([(0.0, 1e-10, 10**6), (0.0, 1e-10, 10**6),
                                             (0.01, 1e-300, 1000)]):
        say(f"single graph replay trial {trial}: shift+{ds} tol={tol} kmax={kmax}")
        rhs = dev(torch, gaussian_vector(b.n, 40 + trial))
        xe, ie = gpu.minres_solve(b, f, sigma + ds, rhs, tol=tol, kmax=kmax, ws=ws_e)
        gpu.apply_H(b, f, sigma, rhs)
        torch.cuda.synchronize()
        xg, ig = gpu.minres_solve(b, f, sigma + ds, rhs, tol=tol, kmax=kmax, ws=ws_g)
        assert ie.iters == ig.iters and ie.phi == ig.phi
        assert torch.equal(xe, xg)
