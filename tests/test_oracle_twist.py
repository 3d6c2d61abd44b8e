"""Pins for the oracle's twist overlap (Sec. III, App. B, App. C)."""
import math

import numpy as np
import pytest

from oracle import model, twist
from workloads import disorder_fields


@pytest.mark.parametrize("L", [4, 6, 8, 10, 12, 14, 16])
def test_phase_sum_vanishes(L):
    """Lemma of App. B."""
    u = twist.twist_phases(L)
    assert abs(u.sum()) < 1e-12 * math.comb(L, L // 2)
    assert np.allclose(np.abs(u), 1.0)


def test_phases_against_kronecker_exponential():
    """u_alpha from the matrix exponential of the full-space operator."""
    L = 6
    from scipy.linalg import expm
    Zop = sum(j * model._site_op(model._SZ, j, L) for j in range(1, L + 1))
    U = expm(1j * 2 * np.pi / L * Zop)
    st = model.sector_states(L)
    assert np.allclose(np.diag(U)[st], twist.twist_phases(L), atol=1e-13)
    assert np.abs(U - np.diag(np.diag(U))).max() < 1e-13


def _eig(L, h):
    return np.linalg.eigh(model.hamiltonian_dense(L, h))


@pytest.mark.parametrize("L", [8, 10])
def test_symmetries_of_z(L):
    h = disorder_fields(L, 3.0, 9)
    w, V = _eig(L, h)
    z = twist.twist_overlap(L, V)
    assert np.all(np.abs(z) <= 1 + 1e-14)
    # translation: T^dagger U T = -U (App. B) -> z(roll h) = -z(h)
    w2, V2 = _eig(L, np.roll(h, 1))
    z2 = twist.twist_overlap(L, V2)
    # reflection and spin flip conjugate z
    z3 = twist.twist_overlap(L, _eig(L, h[::-1])[1])
    z4 = twist.twist_overlap(L, _eig(L, -h)[1])
    gaps = np.diff(w)
    ok = np.ones(len(w), bool)
    ok[:-1] &= gaps > 1e-8
    ok[1:] &= gaps > 1e-8
    assert np.abs(z2 + z)[ok].max() < 1e-9
    assert np.abs(z3 - np.conj(z))[ok].max() < 1e-9
    assert np.abs(z4 - np.conj(z))[ok].max() < 1e-9


@pytest.mark.parametrize("L", [8, 12])
def test_twist_energy_identity_and_bound(L):
    """<U psi|H|U psi> - <psi|H|psi> = (cos(2 pi/L) - 1) <psi|H_xy|psi> for real
    psi, bounded by pi^2/L (Sec. III)."""
    h = disorder_fields(L, 2.0, 4)
    H = model.hamiltonian_dense(L, h)
    Hxy = model.hamiltonian_xy_csr(L).toarray()
    _, V = np.linalg.eigh(H)
    for i in (0, V.shape[1] // 2, V.shape[1] - 1):
        psi = V[:, i]
        Up = twist.twist_state(L, psi)
        dE = np.real(np.conj(Up) @ (H @ Up)) - psi @ H @ psi
        assert abs(dE - (math.cos(2 * math.pi / L) - 1) * (psi @ Hxy @ psi)) < 1e-12
        assert abs(dE) <= math.pi ** 2 / L


def test_gaussian_mean_abs_z2_is_2_over_n():
    """The Gaussian-state value of Sec. III (App. B): mean |z|^2 = 2/n for Gaussian c_alpha."""
    L = 10
    n = math.comb(L, L // 2)
    rng = np.random.default_rng(123)
    c = rng.standard_normal((n, 4000)) / math.sqrt(n)
    z2 = np.abs(twist.twist_overlap(L, c)) ** 2
    mean, se = z2.mean(), z2.std() / math.sqrt(z2.size)
    assert abs(mean - 2.0 / n) < 4 * se


def _perturbative_check(L, hs):
    """Largest |z - z_pred| / |z_pred - u_alpha| and largest |z - u_alpha| / bound
    over all eigenstates, with z_pred the second-order expression of App. C."""
    h = disorder_fields(L, hs, 2)
    H = model.hamiltonian_dense(L, h)
    _, V = np.linalg.eigh(H)
    st = model.sector_states(L)
    d0 = model.diagonal(L, h, st) - model.diagonal(L, np.zeros(L), st)   # H0 = -sum h_j S^z_j
    u = twist.twist_phases(L, st)
    Voff = model.hamiltonian_xy_csr(L).toarray()
    worst_pred = worst_bound = 0.0
    for i in range(V.shape[1]):
        a = int(np.argmax(np.abs(V[:, i])))
        den = d0[a] - d0
        den[a] = np.inf
        c1 = Voff[:, a] / den                       # first-order coefficients
        n2 = np.sum(c1 ** 2)
        z = twist.twist_overlap(L, V[:, i])         # normalised state
        pred = (u[a] + np.sum(c1 ** 2 * u)) / (1 + n2)
        worst_pred = max(worst_pred, abs(z - pred) / abs(pred - u[a]))
        worst_bound = max(worst_bound, abs(z - u[a]) / (2 * math.sin(math.pi / L) * n2 / (1 + n2)))
    return worst_pred, worst_bound


def test_localized_perturbative_bound():
    """The perturbative bound of Sec. III (App. C): the bound holds up to O(J^3), so
    the relative excess and the error of the second-order expression shrink
    like J/h as the disorder grows."""
    p1, b1 = _perturbative_check(8, 400.0)
    p2, b2 = _perturbative_check(8, 1600.0)
    assert p2 < 0.03 and b2 < 1.01
    assert 3.0 < p1 / p2 < 5.5           # O(J^3)/O(J^2) ~ 1/h
    assert (b1 - 1) / (b2 - 1) > 3.0
