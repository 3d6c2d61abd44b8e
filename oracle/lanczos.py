"""Shift-invert Lanczos (Sec. II, Alg. 1) and the eigenpairs it converges to.

``eigenpairs_dense`` is the definition: the nev eigenpairs of H whose
eigenvalues are closest to sigma, from a dense symmetric eigensolver.
Selection and output order: smallest |E - sigma| first (ties to the lower E),
returned in ascending E. The sign of each eigenvector is fixed so that its
largest-magnitude entry (lowest index on ties) is positive.

``si_lanczos`` takes the steps of Alg. 1 in order: solve (A - sigma I) x = v_k,
three-term orthogonalisation giving alpha_k, normalisation giving beta_{k+1},
stop on beta_{k+1} = 0 or k = m, then the Ritz pairs sigma + 1/theta_i and
V_k y_i from the tridiagonal T_k. Full reorthogonalisation of w against
v_1..v_k (Fig. 1 caption) is two passes of classical Gram-Schmidt. The
optional convergence test stops early once the nev Ritz values of largest
|theta| have residual estimates below the requested bound (the paper states
no stopping rule besides beta = 0 or k = m).

``extremal_eigenvalues`` gives E_min and E_max, which fix
sigma = (E_min + E_max) / 2 (Sec. IV A).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def fix_sign(vecs: np.ndarray) -> np.ndarray:
    vecs = np.array(vecs, dtype=np.float64, copy=True)
    if vecs.ndim == 1:
        vecs = vecs[:, None]
    for i in range(vecs.shape[1]):
        a = np.abs(vecs[:, i])
        k = int(np.argmax(a))  # first index among maxima
        if vecs[k, i] < 0:
            vecs[:, i] = -vecs[:, i]
    return vecs


def select_nearest(evals: np.ndarray, sigma: float, nev: int) -> np.ndarray:
    """Indices of the nev eigenvalues closest to sigma (ties to lower E),
    returned so that the selected eigenvalues are ascending."""
    order = np.lexsort((evals, np.abs(evals - sigma)))
    chosen = order[:nev]
    return chosen[np.argsort(evals[chosen], kind="stable")]


def eigenpairs_dense(H: np.ndarray, sigma: float, nev: int):
    w, V = np.linalg.eigh(H)
    idx = select_nearest(w, sigma, nev)
    return w[idx], fix_sign(V[:, idx])


def eigenpairs_shift_invert_sparse(H: sp.spmatrix, sigma: float, nev: int):
    """ARPACK shift-invert with a sparse LU (library routine), for sizes where
    a dense eigensolver is too large."""
    w, V = spla.eigsh(H.tocsc(), k=nev, sigma=sigma, which="LM", tol=0)
    idx = np.argsort(w)
    return w[idx], fix_sign(V[:, idx])


def extremal_eigenvalues(H) -> tuple[float, float]:
    if sp.issparse(H) and H.shape[0] > 4000:
        lo = spla.eigsh(H, k=1, which="SA", tol=1e-14)[0][0]
        hi = spla.eigsh(H, k=1, which="LA", tol=1e-14)[0][0]
        return float(lo), float(hi)
    w = np.linalg.eigvalsh(H.toarray() if sp.issparse(H) else H)
    return float(w[0]), float(w[-1])


def sigma_midpoint(H) -> float:
    emin, emax = extremal_eigenvalues(H)
    return 0.5 * (emin + emax)


def si_lanczos(solve, v: np.ndarray, m: int, sigma: float, nev: int | None = None,
               hnorm: float = 1.0, eig_tol: float = 0.0):
    """Alg. 1. ``solve(v)`` returns (A - sigma I)^{-1} v.

    Returns dict with Ritz values (all k, ascending in theta), the selected
    nev pairs (eigenvalue ascending), alpha, beta and the step count.
    With ``eig_tol > 0`` the loop also stops once every selected pair's
    estimate hnorm * |beta_{k+1} y_{k,i}| / |theta_i| is <= eig_tol * hnorm.
    """
    n = v.shape[0]
    V = np.zeros((n, m), dtype=np.float64)
    alphas, betas = [], []
    beta = np.linalg.norm(v)            # beta_1
    v_prev = np.zeros(n)
    vk = v / beta
    k = 0
    beta_next = 0.0
    while True:
        k += 1
        V[:, k - 1] = vk
        x = solve(vk)
        w = x - beta * v_prev
        alpha = vk @ w
        w = w - alpha * vk
        for _ in range(2):               # full reorthogonalisation (CGS2)
            Vk = V[:, :k]
            w = w - Vk @ (Vk.T @ w)
        beta_next = np.linalg.norm(w)
        alphas.append(alpha)
        betas.append(beta_next)
        if nev is not None and eig_tol > 0 and k >= nev:
            theta, Y = _tridiag_eig(alphas, betas[:-1])
            sel = np.argsort(-np.abs(theta))[:nev]
            est = hnorm * np.abs(beta_next * Y[-1, sel]) / np.abs(theta[sel])
            if np.all(est <= eig_tol * hnorm):
                break
        if beta_next == 0.0 or k == m:
            break
        v_prev = vk
        vk = w / beta_next
        beta = beta_next
    theta, Y = _tridiag_eig(alphas, betas[:-1])
    lam = sigma + 1.0 / theta
    out = dict(theta=theta, lam=lam, steps=k, alpha=np.array(alphas), beta=np.array(betas))
    if nev is not None:
        sel = np.argsort(-np.abs(theta))[:nev]
        sel = sel[np.argsort(lam[sel])]
        out["evals"] = lam[sel]
        out["evecs"] = fix_sign(V[:, :k] @ Y[:, sel])
    return out


def _tridiag_eig(alphas, offdiag):
    k = len(alphas)
    T = np.diag(np.asarray(alphas, dtype=np.float64))
    if k > 1:
        o = np.asarray(offdiag, dtype=np.float64)
        T += np.diag(o, 1) + np.diag(o, -1)
    return np.linalg.eigh(T)


def eigen_residuals(H, evals, evecs) -> np.ndarray:
    """||H psi_i - E_i psi_i||_2 for each pair."""
    R = H @ evecs - evecs * np.asarray(evals)[None, :]
    return np.linalg.norm(R, axis=0)
