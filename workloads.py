"""Seeded synthetic inputs for the random-field Heisenberg chain.

This module holds no arithmetic of the method. It only draws the random
numbers that the problem statement asks for, so that the CPU oracle and the
HIP path receive identical inputs:

* disorder fields h_j, i.i.d. uniform on [-h, h] (Sec. I, below Eq. (1));
* Lanczos start vectors and test vectors (Gaussian, unnormalised);
* the meta draw (chain length L_r and disorder strength h_r) of a batch of
  realizations.

Every generator is NumPy's PCG64 through ``numpy.random.default_rng(seed)``.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

# Offset of the seed stream used for the batched meta draw, kept apart from
# the field seeds 0, 1, 2, ... so that the two never share a stream.
META_SEED_OFFSET = 10**6


def disorder_fields(L: int, h: float, seed: int) -> np.ndarray:
    """h_1..h_L drawn i.i.d. from U[-h, h] (Sec. I)."""
    return np.random.default_rng(seed).uniform(-h, h, L).astype(np.float64)


def gaussian_vector(n: int, seed: int) -> np.ndarray:
    """Unnormalised standard-normal FP64 vector of length n."""
    return np.random.default_rng(seed).standard_normal(n).astype(np.float64)


def start_vector(n: int, seed: int) -> np.ndarray:
    """Lanczos start vector v (Alg. 1 normalises it itself)."""
    return gaussian_vector(n, 10_000 + seed)


@dataclass(frozen=True)
class Realization:
    index: int
    L: int
    h: float
    fields: np.ndarray


def batched_realization(r: int, Ls=(14, 16, 18), hs=(2.0, 3.0, 4.0)) -> Realization:
    """Realization r of a mixed-size batch: L_r and h_r from a meta stream,
    then the fields h_j ~ U[-h_r, h_r] from seed r."""
    m = np.random.default_rng(META_SEED_OFFSET + r)
    L = int(m.choice(np.asarray(Ls)))
    h = float(m.choice(np.asarray(hs)))
    return Realization(r, L, h, disorder_fields(L, h, r))


def batched_realizations(count: int, **kw) -> list[Realization]:
    return [batched_realization(r, **kw) for r in range(count)]


# The five workloads the method is exercised on, by what they are.
WORKLOADS = {
    "plain_L14": dict(L=14, h=3.0, seeds=[0], nev=10, minres_tol=1e-12),
    "batched_L14_16_18": dict(Ls=(14, 16, 18), hs=(2.0, 3.0, 4.0), count=512, nev=6, minres_tol=1e-12),
    "mixed_L22": dict(L=22, h=3.5, seeds=list(range(32)), nev=20, minres_tol=1e-12),
    "grad_L20": dict(L=20, h=3.0, seeds=list(range(16)), nev=4, minres_tol=1e-12),
    "largest_L26": dict(L=26, h=3.8, seeds=[0], nev=10, minres_tol=1e-12),
}
