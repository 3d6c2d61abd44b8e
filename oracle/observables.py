"""Eigenstate observables of Sec. IV (entanglement and level spacing).

* ``entanglement_entropy``: the bipartite entropy S = -Tr rho_A ln rho_A of
  a sector vector, with rho_A the reduced density matrix of subsystem A =
  sites 1..la (the paper takes la = L/2). It is the Schmidt decomposition
  written out: the vector is placed on the full 2^L basis, reshaped into the
  (B, A) coefficient matrix, and its squared singular values, normalised to
  sum 1, are the eigenvalues of rho_A.
* ``spacing_ratios``: r_k = min(delta_k, delta_{k-1}) / max(delta_k,
  delta_{k-1}) with delta_k = E_{k+1} - E_k over the sorted eigenvalues.
* ``rmt_entropy``: the random-matrix estimate of S quoted in Sec. IV,
  the random-state entropy of Sec. IV B, as a reference curve (not a pin).

Readings where the paper is silent:
* the logarithm is natural (the reference values use ln 2);
* the vector is normalised inside (Tr rho_A = 1 for any input scale);
* a ratio whose two spacings are both zero is undefined: it is NaN and left
  out of the mean.

TEST INFRASTRUCTURE ONLY (see the package docstring).
"""
from __future__ import annotations

import numpy as np

from .model import sector_states


def schmidt_probabilities(L: int, psi: np.ndarray, la: int) -> np.ndarray:
    """Eigenvalues of rho_A (A = sites 1..la = bits 0..la-1), descending."""
    if not 1 <= la <= L - 1:
        raise ValueError("la must be in 1..L-1")
    psi = np.asarray(psi, dtype=np.float64)
    full = np.zeros(1 << L, dtype=np.float64)
    full[sector_states(L)] = psi
    # state = b * 2^la + a, with a the bits of sites 1..la
    mat = full.reshape(1 << (L - la), 1 << la)
    s = np.linalg.svd(mat, compute_uv=False)
    p = s ** 2
    return p / p.sum()


def entanglement_entropy(L: int, psi: np.ndarray, la: int | None = None) -> float:
    """S = -sum_i p_i ln p_i over the Schmidt probabilities (0 ln 0 = 0)."""
    p = schmidt_probabilities(L, psi, L // 2 if la is None else la)
    p = p[p > 0]
    return float(-(p * np.log(p)).sum())


def spacing_ratios(E: np.ndarray) -> np.ndarray:
    """r_k for k = 1..len(E)-2 of the sorted eigenvalues."""
    E = np.sort(np.asarray(E, dtype=np.float64))
    d = np.diff(E)
    lo = np.minimum(d[1:], d[:-1])
    hi = np.maximum(d[1:], d[:-1])
    with np.errstate(invalid="ignore", divide="ignore"):
        r = lo / hi
    r[hi == 0] = np.nan
    return r


def mean_spacing_ratio(E: np.ndarray) -> float:
    r = spacing_ratios(E)
    return float(np.nanmean(r)) if np.isfinite(r).any() else float("nan")


def rmt_entropy(L: int) -> float:
    """The random-state entropy of Sec. IV B: (ln 2 / 2) L + (1/2) ln(1/2) - 1/4."""
    return 0.5 * np.log(2.0) * L + 0.5 * np.log(0.5) - 0.25
