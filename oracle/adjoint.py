"""Derivatives of an eigenpair with respect to the fields h_j.

dH/dh_j = -S^z_j (Eq. (1)), which is diagonal with entries -s_j(alpha).

* Hellmann-Feynman: dE_n/dh_j = <psi_n| dH/dh_j |psi_n> = -sum_alpha c_alpha^2 s_j(alpha).
* First-order perturbation sum for the eigenvector (non-degenerate E_n):
  d psi_n/dh_j = sum_{m != n} psi_m <psi_m| dH/dh_j |psi_n> / (E_n - E_m).
* z = sum_alpha c_alpha^2 u_alpha (App. B), so
  dz/dh_j = 2 sum_alpha c_alpha (dc_alpha/dh_j) u_alpha and
  d|z|^2/dh_j = 2 Re(conj(z) dz/dh_j).

Both need the full spectrum, so this is for small L only.
"""
from __future__ import annotations

import numpy as np

from .model import hamiltonian_dense, sector_states, spin
from .twist import twist_phases


def spin_matrix(L: int) -> np.ndarray:
    """s_j(alpha) for all states (rows) and sites j = 1..L (columns)."""
    st = sector_states(L)
    return np.stack([spin(st, j) for j in range(1, L + 1)], axis=1)


def hellmann_feynman(L: int, psi: np.ndarray) -> np.ndarray:
    """dE/dh_j = -<S^z_j> for a real normalised psi."""
    return -(psi ** 2) @ spin_matrix(L)


def eigvec_derivatives(L: int, h: np.ndarray, n_index: int):
    """(E, psi, dpsi) with dpsi[:, j] = d psi / dh_{j+1} by the perturbation
    sum over the full dense spectrum."""
    H = hamiltonian_dense(L, h)
    w, V = np.linalg.eigh(H)
    S = spin_matrix(L)
    psi = V[:, n_index]
    E = w[n_index]
    dpsi = np.zeros((H.shape[0], L))
    denom = E - w
    denom[n_index] = np.inf
    for j in range(L):
        coup = V.T @ (-S[:, j] * psi)           # <psi_m| dH/dh_j |psi_n>
        dpsi[:, j] = V @ (coup / denom)
    return E, psi, dpsi


def dz2_dh(L: int, psi: np.ndarray, dpsi: np.ndarray) -> np.ndarray:
    u = twist_phases(L)
    z = np.sum(psi ** 2 * u)
    dz = 2.0 * ((psi * u)[:, None] * dpsi).sum(axis=0)
    return 2.0 * np.real(np.conj(z) * dz)


def finite_difference(L: int, h: np.ndarray, target_E: float, step: float = 1e-5):
    """Central differences of E and |z|^2 for the eigenpair whose eigenvalue is
    nearest ``target_E`` (re-identified in the perturbed spectra)."""
    u = twist_phases(L)

    def pair(hh):
        w, V = np.linalg.eigh(hamiltonian_dense(L, hh))
        i = int(np.argmin(np.abs(w - target_E)))
        psi = V[:, i]
        return w[i], abs(np.sum(psi ** 2 * u)) ** 2

    dE = np.zeros(L)
    dz2 = np.zeros(L)
    for j in range(L):
        hp = np.array(h, dtype=np.float64)
        hm = hp.copy()
        hp[j] += step
        hm[j] -= step
        Ep, zp = pair(hp)
        Em, zm = pair(hm)
        dE[j] = (Ep - Em) / (2 * step)
        dz2[j] = (zp - zm) / (2 * step)
    return dE, dz2
