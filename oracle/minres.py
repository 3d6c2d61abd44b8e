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

    Each iteration has three parts, taken in the paper's order:

    1. the preconditioned Lanczos recurrence: with q_k = M^{-1} z_k and
       beta_k = sqrt(q_k . z_k), the vectors q_k / beta_k are M-orthonormal and
       A (q_k / beta_k) = beta_{k+1} q_{k+1} / beta_{k+1} + alpha_k q_k / beta_k
       + beta_k q_{k-1} / beta_{k-1}, i.e. A is tridiagonal (T_k) in that basis;
    2. one Givens rotation more in the QR factorisation of T_k: the previous
       rotation (c, s) acting on the new column gives delta_k and gamma-hat_k
       and the entries it pushes down (epsilon_{k+1}, delta-hat_{k+1}); the new
       rotation annihilates beta_{k+1} below gamma-hat_k;
    3. the search direction d_k = (q_k / beta_k - delta_k d_{k-1} -
       epsilon_k d_{k-2}) / gamma_k (the columns of V_k R_k^{-1}) and the
       step x += tau_k d_k, with tau_k = c_k phi_{k-1}; phi_k = -s_k phi_{k-1}
       is the rotated right-hand side, |phi_k| the residual norm.

    Returns (x, k, phi_history).
    """
    def precondition(v):
        return minv_diag * v

    # Lanczos vectors: z_{k-1}, z_k, q_k, and beta_{k-1}, beta_k
    z_old = np.zeros_like(b)
    z = b - matvec(x0)
    q = precondition(z)
    beta_old, beta = 1.0, np.sqrt(q @ z)
    # QR state: the last rotation and the entries it carries to the next column
    c_rot, s_rot = 1.0, 0.0
    dhat, eps = 0.0, 0.0
    phi = beta
    # search directions d_{k-1}, d_{k-2} and the iterate
    d1 = np.zeros_like(b)
    d2 = np.zeros_like(b)
    x = x0.astype(np.float64).copy()
    k = 0
    hist = [abs(phi)]
    while abs(phi) >= tol and k < kmax:
        k += 1
        # 1. Lanczos: alpha_k and the next (z, q, beta)
        p = matvec(q)
        alpha = (q @ p) / beta ** 2
        z_new = p / beta - (alpha / beta) * z - (beta / beta_old) * z_old
        q_new = precondition(z_new)
        beta_new = np.sqrt(q_new @ z_new)
        # 2. QR of T_k: old rotation on the new column, then the new rotation
        delta = c_rot * dhat + s_rot * alpha
        gamma_hat = -s_rot * dhat + c_rot * alpha
        eps_new = s_rot * beta_new
        dhat_new = c_rot * beta_new
        gamma = np.sqrt(gamma_hat ** 2 + beta_new ** 2)
        c_rot, s_rot = gamma_hat / gamma, beta_new / gamma
        tau = c_rot * phi
        phi = -s_rot * phi
        # 3. search direction and step
        d = (q / beta - delta * d1 - eps * d2) / gamma
        x = x + tau * d
        # shift the recurrences by one
        z_old, z, q = z, z_new, q_new
        beta_old, beta = beta, beta_new
        dhat, eps = dhat_new, eps_new
        d2, d1 = d1, d
        hist.append(abs(phi))
    return x, k, np.asarray(hist)


def solve_dense(A: np.ndarray, sigma: float, b: np.ndarray) -> np.ndarray:
    """x = (A - sigma I)^{-1} b by LAPACK: what MINRES converges to."""
    n = A.shape[0]
    return np.linalg.solve(A - sigma * np.eye(n), b)
