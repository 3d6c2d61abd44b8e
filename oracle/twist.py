"""The twist operator and the twist overlap (Sec. III, App. B).

U_twist = exp[i 2 pi / L sum_{j=1}^{L} j S^z_j] is diagonal in the S^z basis,
with u_alpha = <alpha|U_twist|alpha>. For a real eigenvector with
coefficients c_alpha, z = <psi|U_twist|psi> = sum_alpha c_alpha^2 u_alpha.
"""
from __future__ import annotations

import numpy as np

from .model import sector_states, spin


def twist_phases(L: int, states: np.ndarray | None = None) -> np.ndarray:
    """u_alpha = exp(i 2 pi / L * sum_j j s_j(alpha)), evaluated directly."""
    if states is None:
        states = sector_states(L)
    arg = np.zeros(states.shape[0], dtype=np.float64)
    for j in range(1, L + 1):
        arg += j * spin(states, j)
    return np.exp(1j * 2.0 * np.pi / L * arg)


def twist_overlap(L: int, psi: np.ndarray) -> np.ndarray:
    """z for each column of psi (real coefficients)."""
    u = twist_phases(L)
    psi = np.asarray(psi, dtype=np.float64)
    if psi.ndim == 1:
        return np.sum(psi ** 2 * u)
    return (psi ** 2 * u[:, None]).sum(axis=0)


def twist_state(L: int, psi: np.ndarray) -> np.ndarray:
    """U_twist |psi> (complex)."""
    return twist_phases(L) * psi
