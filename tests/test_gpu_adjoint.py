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
