"""Eigenpair derivatives on the GPU (Hellmann-Feynman and the adjoint MINRES
solve) against the CPU oracle's perturbation sum and finite differences."""
import sys

import numpy as np
import pytest

from oracle import adjoint, lanczos, model
from workloads import disorder_fields, start_vector

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


@pytest.mark.parametrize("L,seed,nev", [(10, 1, 3), (12, 2, 4)])
def test_eig_grad_matches_perturbation_sum(gpu, torch, L, seed, nev):
    say(f"eig_grad L={L} seed={seed}")
    h = disorder_fields(L, 3.0, seed)
    H = model.hamiltonian_dense(L, h)
    w = np.linalg.eigvalsh(H)
    sigma = 0.5 * (w[0] + w[-1])
    b = gpu.Basis(L)
    res = gpu.si_lanczos(b, h, sigma, nev, v0=torch.as_tensor(start_vector(b.n, 1), device="cuda"))
    assert res.nconv == nev
    for t in range(nev):
        E = res.evals[t]
        psi = res.evecs[:, t].contiguous()
        dE, dz2, z, info = gpu.eig_grad(b, h, E, psi, tol=1e-11)
        k = int(np.argmin(np.abs(w - E)))
        E_ref, psi_ref, dpsi = adjoint.eigvec_derivatives(L, h, k)
        dE_ref = adjoint.hellmann_feynman(L, psi_ref)
        dz2_ref = adjoint.dz2_dh(L, psi_ref, dpsi)
        gap = np.min(np.abs(np.delete(w, k) - E_ref))
        say(f"  pair {t}: gap={gap:.2e} minres={info.iters} |dE err|={np.abs(dE - dE_ref).max():.2e} "
            f"|dz2 err|={np.abs(dz2 - dz2_ref).max():.2e}")
        # Hellmann-Feynman is exact for the computed psi; its error is
        # O(||psi - psi_ref||) = O(residual / gap) with residual <= 1e-10 ||H||
        assert np.abs(dE - dE_ref).max() <= 5e-10
        # adjoint solve to 1e-11 in the M^-1 norm; error amplified by ~1/gap
        assert np.abs(dz2 - dz2_ref).max() <= 1e-7 * max(1.0, np.abs(dz2_ref).max())
        assert abs(dE.sum()) <= 1e-11 and abs(dz2.sum()) <= 1e-8 * max(1.0, np.abs(dz2).max())


def test_eig_grad_vs_finite_differences(gpu, torch):
    say("eig_grad vs FD L=10")
    L = 10
    h = disorder_fields(L, 3.0, 4)
    H = model.hamiltonian_dense(L, h)
    w = np.linalg.eigvalsh(H)
    sigma = 0.5 * (w[0] + w[-1])
    b = gpu.Basis(L)
    res = gpu.si_lanczos(b, h, sigma, 1, v0=torch.as_tensor(start_vector(b.n, 2), device="cuda"))
    E = res.evals[0]
    dE, dz2, _, _ = gpu.eig_grad(b, h, E, res.evecs[:, 0].contiguous(), tol=1e-12)
    dE_fd, dz2_fd = adjoint.finite_difference(L, h, E, step=1e-5)
    assert np.abs(dE - dE_fd).max() <= 1e-6
    assert np.abs(dz2 - dz2_fd).max() <= 1e-5 * max(1.0, np.abs(dz2).max())


def test_autograd_eigpair(gpu, torch):
    say("autograd EigPair L=10")
    L = 10
    h = disorder_fields(L, 3.0, 6)
    H = model.hamiltonian_dense(L, h)
    w = np.linalg.eigvalsh(H)
    sigma = 0.5 * (w[0] + w[-1])
    b = gpu.Basis(L)
    fn = gpu.EigPair(b, sigma, nev=2, which=1, v0=torch.as_tensor(start_vector(b.n, 3), device="cuda"))
    ht = torch.tensor(h, dtype=torch.float64, requires_grad=True)
    E, z2 = fn(ht)
    (0.3 * E + 2.0 * z2).backward()
    E_sel, _ = lanczos.eigenpairs_dense(H, sigma, 2)
    k = int(np.argmin(np.abs(w - E_sel[1])))
    _, psi, dpsi = adjoint.eigvec_derivatives(L, h, k)
    ref = 0.3 * adjoint.hellmann_feynman(L, psi) + 2.0 * adjoint.dz2_dh(L, psi, dpsi)
    assert abs(E.item() - E_sel[1]) <= 1e-10
    assert np.abs(ht.grad.numpy() - ref).max() <= 1e-7 * max(1.0, np.abs(ref).max())


def _inverse_iteration(gpu, torch, b, h, E, psi, steps=3, tol=1e-9):
    """Eigenvector of H(h) nearest E by inverse iteration from psi: each step
    solves (H - E) y = v with MINRES and normalises (the perturbed eigenvalue
    is within ~1e-7 of E, so each step shrinks the other components by
    ~1e-7 / gap)."""
    v = psi / torch.linalg.norm(psi)
    for _ in range(steps):
        y, _info = gpu.minres_solve(b, h, E, v.contiguous(), tol=tol, kmax=40 * b.n)
        v = y / torch.linalg.norm(y)
    if float(torch.dot(v, psi)) < 0:
        v = -v
    return v


def _fd_subset(gpu, torch, L, seeds, sites, delta=1e-7):
    """Adjoint derivatives of the eigenpair nearest sigma against central
    finite differences, the perturbed eigenpairs found by inverse iteration
    seeded from psi with shift E (Rayleigh quotient for E', twist of psi' for
    z'). Returns the largest deviations."""
    worst_E, worst_z = 0.0, 0.0
    for seed in seeds:
        h = disorder_fields(L, 3.0, seed)
        b = gpu.Basis(L)
        lo, hi, sg = gpu.sigma_midpoint(b, h, 1e-12)
        res = gpu.si_lanczos(b, h, sg, 2, escale=max(abs(lo), abs(hi)),
                             v0=torch.as_tensor(start_vector(b.n, seed), device="cuda"))
        assert res.nconv == 2
        t = int(np.argmin(np.abs(res.evals - sg)))
        E = res.evals[t]
        psi = res.evecs[:, t].contiguous()
        gap = float(np.min(np.abs(np.delete(res.evals, t) - E)))
        dE, dz2, z, info = gpu.eig_grad(b, h, E, psi, tol=1e-12)
        assert abs(dE.sum()) <= 1e-10 and abs(dz2.sum()) <= 1e-7 * max(1.0, np.abs(dz2).max())
        for j in sites:
            Ep, z2p = [], []
            for sgn in (1.0, -1.0):
                hp = h.copy()
                hp[j] += sgn * delta
                v = _inverse_iteration(gpu, torch, b, hp, E, psi)
                Ep.append(float(torch.dot(v, gpu.apply_H(b, hp, 0.0, v))))
                z2p.append(abs(gpu.twist_expect(b, v)[0]) ** 2)
            dE_fd = (Ep[0] - Ep[1]) / (2 * delta)
            dz2_fd = (z2p[0] - z2p[1]) / (2 * delta)
            eE, ez = abs(dE[j] - dE_fd), abs(dz2[j] - dz2_fd) / max(1.0, abs(dz2[j]))
            say(f"  L={L} seed={seed} site={j + 1} gap>={gap:.1e} dE={dE[j]:+.9f} fd={dE_fd:+.9f} "
                f"dz2={dz2[j]:+.6e} fd={dz2_fd:+.6e} minres={info.iters}")
            worst_E, worst_z = max(worst_E, eE), max(worst_z, ez)
    return worst_E, worst_z


def test_eig_grad_fd_by_inverse_iteration_L18(gpu, torch):
    """Derivatives of a mid-spectrum eigenpair at L=18 against finite
    differences of eigenpairs obtained without the adjoint code. Step 1e-7:
    the central-difference error is ~ delta^2 |V|^3 / gap^2 for E and
    ~ delta^2 |V|^3 / gap^3 relative to d|z|^2/dh ~ |V| / gap for |z|^2,
    both below the tolerances for gaps >= 1e-4; rounding of E' (~1e-13)
    divided by 2 delta gives ~1e-6."""
    say("eig_grad vs FD by inverse iteration, L=18")
    eE, ez = _fd_subset(gpu, torch, 18, seeds=(0,), sites=(0, 7, 12))
    assert eE <= 2e-5
    assert ez <= 1e-3
