"""Preconditioned MINRES (App. A, Alg. 2) and its plain definition.

``minres`` takes the steps of Alg. 2 in the paper's order and notation:
a preconditioned Lanczos three-term recurrence on z_k with q_k = M^{-1} z_k,
a Givens rotation that eliminates the subdiagonal, and the search-direction
recurrence for d_k. It returns x_k and the history of |phi_k|, where
|phi_k| = ||b - A x_k||_{M^{-1}} is the preconditioned residual norm.

Readings where the algorithm leaves something open:
* epsilon_1 is used in the first d-update but never set; it multiplies
  d_{-1} = 0, so it is taken as 0;
* the stopping test is the printed absolute test |phi_k| < tolerance.

``solve_dense`` is the definition of what MINRES converges to.
"""
from __future__ import annotations

import numpy as np


def minres(matvec, x0: np.ndarray, b: np.ndarray, minv_diag: np.ndarray,
           kmax: int, tol: float):
    """Alg. 2. ``matvec(v)`` applies A; ``minv_diag`` is the diagonal of M^{-1}.

    Returns (x, k, phi_history).
    """
    Minv = lambda v: minv_diag * v  # noqa: E731
    z_prev = np.zeros_like(b)
    z = b - matvec(x0)
    q = Minv(z)
    beta_prev = 1.0
    beta = np.sqrt(q @ z)
    phi = beta
    dhat = 0.0
    c_prev, s_prev = 1.0, 0.0
    d_prev2 = np.zeros_like(b)
    d_prev = np.zeros_like(b)
    eps = 0.0
    x = x0.astype(np.float64).copy()
    k = 0
    hist = [abs(phi)]
    while abs(phi) >= tol and k < kmax:
        k += 1
        p = matvec(q)
        alpha = (q @ p) / beta ** 2
        z_next = p / beta - (alpha / beta) * z - (beta / beta_prev) * z_prev
        q_next = Minv(z_next)
        beta_next = np.sqrt(q_next @ z_next)
        delta = c_prev * dhat + s_prev * alpha
        gamma_hat = -s_prev * dhat + c_prev * alpha
        eps_next = s_prev * beta_next
        dhat_next = c_prev * beta_next
        gamma = np.sqrt(gamma_hat ** 2 + beta_next ** 2)
        c = gamma_hat / gamma
        s = beta_next / gamma
        tau = c * phi
        phi = -s * phi
        d = (q / beta - delta * d_prev - eps * d_prev2) / gamma
        x = x + tau * d
        # advance the recurrences
        z_prev, z = z, z_next
        q = q_next
        beta_prev, beta = beta, beta_next
        dhat, eps = dhat_next, eps_next
        c_prev, s_prev = c, s
        d_prev2, d_prev = d_prev, d
        hist.append(abs(phi))
    return x, k, np.asarray(hist)


def solve_dense(A: np.ndarray, sigma: float, b: np.ndarray) -> np.ndarray:
    """x = (A - sigma I)^{-1} b by LAPACK: what MINRES converges to."""
    n = A.shape[0]
    return np.linalg.solve(A - sigma * np.eye(n), b)
