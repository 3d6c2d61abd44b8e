"""Shift-invert Lanczos on the row-launch MINRES path against the oracle.

At L >= 16 the MINRES inner solves run as two row launches per iteration,
replayed as captured graphs (the single cooperative kernel only serves grids
of at most 32 workgroups: L <= 14). These tests run the whole path there:

* L = 16 and 18, h = 3, seed 0, nev = 6, FP64 and FP32-inner MINRES. The
  oracle eigenvalues, gaps and twist overlaps are stored values written by
  tests/golden/make_golden.py from the oracle's sparse shift-invert solver
  (about 20 minutes at L = 18, too slow to repeat here). At run time the
  oracle's own CSR matrix gives the explicit residual r_i of each GPU pair,
  and the angle to the exact eigenvector obeys sin(theta_i) <= r_i / delta_i
  (Davis-Kahan), delta_i the distance from E_i to the other eigenvalues
  (stored). The overlap bar 1 - |<u, u_ref>| <= 1e-10 then follows from
  1 - cos(theta_i) <= 1 - sqrt(1 - (r_i / delta_i)^2) <= 1e-10, and
  |z - z_ref| <= 2 ||u - u_ref|| <= 2 sqrt(2 - 2 cos(theta_i)).
* L = 20, h = 3, seed 0, nev = 2 (no stored reference): sigma and the
  extremes against the oracle's sparse Lanczos, the residual with the
  oracle's CSR matrix, and two more GPU runs on the translated fields
  roll(h, 1) and the reflected fields h[::-1] with other start vectors.
  Their spectra equal the first run's; their eigenvectors are the
  translated / reflected first ones (T psi, R psi), for which the App. B
  lemma gives z(T psi) = -z(psi) and z(R psi) = conj z(psi) exactly, so
  |z' + z| <= 2 ||psi' - T psi|| and |z' - conj z| <= 2 ||psi' - R psi||.
  The same eigenpair feeds the L = 20 adjoint check (config 4 subset).
"""
import json
import os
import sys

import numpy as np
import pytest

from oracle import adjoint, lanczos, model, twist
from workloads import disorder_fields, start_vector

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


def _golden(L):
    with open(os.path.join(HERE, "golden", f"si_L{L}_h3_seed0.json")) as fh:
        return json.load(fh)


def _gaps(E, spectrum):
    """Distance from each E_i to the nearest other eigenvalue of the stored
    window (the eigenvalue matched to E_i itself is removed)."""
    spectrum = np.asarray(spectrum)
    out = []
    for e in E:
        k = int(np.argmin(np.abs(spectrum - e)))
        out.append(float(np.min(np.abs(np.delete(spectrum, k) - e))))
    return np.array(out)


@pytest.mark.parametrize("L,prec", [(16, "fp64"), (16, "fp32_inner"), (18, "fp64"),
                                    (18, "fp32_inner")])
def test_si_lanczos_row_path_vs_oracle(gpu, torch, L, prec):
    g = _golden(L)
    f = np.array(g["fields"])
    sigma, nev = g["sigma"], g["nev"]
    escale = max(abs(g["E_min"]), abs(g["E_max"]))
    say(f"si_lanczos row path L={L} {prec} nev={nev}")
    b = gpu.Basis(L)
    v0 = torch.as_tensor(start_vector(b.n, 3), device="cuda")
    res = gpu.si_lanczos(b, f, sigma, nev, escale=escale, v0=v0, precision=prec)
    say(f"  steps={res.steps} minres_iters={res.minres_iters} nconv={res.nconv} "
        f"max_rel={res.max_rel_resid:.2e} t={res.seconds:.1f}s")
    assert res.status == 0 and res.nconv == nev
    Eref = np.array(g["evals"])
    assert np.all(np.abs(res.evals - Eref) / np.maximum(np.abs(Eref), 1) <= 1e-10), res.evals - Eref
    H = model.hamiltonian_csr(L, f)
    U = res.evecs.cpu().numpy()
    r = lanczos.eigen_residuals(H, res.evals, U)
    assert np.all(r <= 1e-10 * escale), r
    assert np.allclose(res.resid, r, rtol=1e-6, atol=1e-14)
    assert np.allclose(np.linalg.norm(U, axis=0), 1.0, atol=1e-12)
    delta = _gaps(res.evals, g["window"])
    sin_bound = np.minimum(1.0, r / delta)
    deficit = 1.0 - np.sqrt(1.0 - sin_bound ** 2)          # bound on 1 - |<u, u_ref>|
    say(f"  residual {r.max():.2e}, min gap {delta.min():.2e}, overlap deficit <= {deficit.max():.2e}")
    assert np.all(deficit <= 1e-10)
    z = gpu.twist_expect(b, res.evecs)
    assert np.abs(z - twist.twist_overlap(L, U)).max() <= 1e-13
    zref = np.array(g["z_re"]) + 1j * np.array(g["z_im"])
    assert np.all(np.abs(z - zref) <= 2 * np.sqrt(2 * deficit) + 1e-12)


def _perm(L, states, f):
    img = np.array([f(int(a)) for a in states], dtype=np.int64)
    p = np.searchsorted(states, img)
    assert np.array_equal(states[p], img)
    return p


def _mapped(U, p):
    out = np.zeros_like(U)
    out[p, :] = U
    return out


@pytest.fixture(scope="module")
def pair_L20(gpu, torch):
    L, nev = 20, 2
    f = disorder_fields(L, 3.0, 0)
    b = gpu.Basis(L)
    say("L=20: sigma and two eigenpairs nearest it")
    emin, emax, sigma = gpu.sigma_midpoint(b, f, 1e-12)
    escale = max(abs(emin), abs(emax))
    res = gpu.si_lanczos(b, f, sigma, nev, escale=escale,
                         v0=torch.as_tensor(start_vector(b.n, 0), device="cuda"))
    say(f"  steps={res.steps} minres_iters={res.minres_iters} nconv={res.nconv} t={res.seconds:.1f}s")
    return dict(L=L, f=f, b=b, emin=emin, emax=emax, sigma=sigma, escale=escale, res=res, nev=nev)


def test_L20_sigma_residual_and_twist_symmetries(gpu, torch, pair_L20):
    P = pair_L20
    L, f, b, nev, res = P["L"], P["f"], P["b"], P["nev"], P["res"]
    H = model.hamiltonian_csr(L, f)
    lo, hi = lanczos.extremal_eigenvalues(H)
    assert abs(P["emin"] - lo) <= 1e-10 * abs(lo) and abs(P["emax"] - hi) <= 1e-10 * abs(hi)
    assert res.status == 0 and res.nconv == nev
    U = res.evecs.cpu().numpy()
    r = lanczos.eigen_residuals(H, res.evals, U)
    say(f"  L=20 evals={res.evals} oracle residuals={r}")
    assert np.all(r <= 1e-10 * P["escale"])
    assert np.allclose(res.resid, r, rtol=1e-6, atol=1e-14)
    z = gpu.twist_expect(b, res.evecs)
    assert np.abs(z - twist.twist_overlap(L, U)).max() <= 1e-13
    states = model.sector_states(L)
    mask = (1 << L) - 1
    maps = {
        "roll": (np.roll(f, 1), lambda a: ((a << 1) | (a >> (L - 1))) & mask, lambda zz: -zz),
        "reverse": (f[::-1].copy(), lambda a: int(format(a, f"0{L}b")[::-1], 2), np.conj),
    }
    for k, (name, (f2, amap, zmap)) in enumerate(maps.items()):
        res2 = gpu.si_lanczos(b, f2, P["sigma"], nev, escale=P["escale"],
                              v0=torch.as_tensor(start_vector(b.n, 11 + k), device="cuda"))
        say(f"  {name}: steps={res2.steps} minres_iters={res2.minres_iters} evals={res2.evals}")
        assert res2.status == 0 and res2.nconv == nev
        # same spectrum (the c16 bar)
        assert np.all(np.abs(res2.evals - res.evals) / np.maximum(np.abs(res.evals), 1) <= 1e-10)
        U2 = res2.evecs.cpu().numpy()
        r2 = lanczos.eigen_residuals(model.hamiltonian_csr(L, f2), res2.evals, U2)
        assert np.all(r2 <= 1e-10 * P["escale"])
        TU = _mapped(U, _perm(L, states, amap))
        dpsi = np.minimum(np.linalg.norm(U2 - TU, axis=0), np.linalg.norm(U2 + TU, axis=0))
        z2 = gpu.twist_expect(b, res2.evecs)
        say(f"    ||psi' - map psi|| = {dpsi}, |z' - map z| = {np.abs(z2 - zmap(z))}")
        # the two runs found the same eigenvectors (converged pairs: r / gap <= ~1e-5 each)
        assert np.all(dpsi <= 1e-4)
        # the lemma of App. B on the device outputs
        assert np.all(np.abs(z2 - zmap(z)) <= 2 * dpsi + 1e-12)


def _inverse_iteration(gpu, torch, b, h, E, psi, steps=3, tol=1e-9):
    v = psi / torch.linalg.norm(psi)
    for _ in range(steps):
        y, _info = gpu.minres_solve(b, h, E, v.contiguous(), tol=tol, kmax=40 * b.n)
        v = y / torch.linalg.norm(y)
    if float(torch.dot(v, psi)) < 0:
        v = -v
    return v


def test_L20_adjoint_vs_finite_differences(gpu, torch, pair_L20):
    """Config 4 subset at full size: L = 20, h = 3, seed 0, the pair nearest
    sigma, sites 1, 10 and 17. Central differences of step 1e-7 of eigenpairs
    found by inverse iteration (no adjoint code); truncation ~ delta^2 / gap^2
    as in the L = 18 test."""
    P = pair_L20
    b, f, res = P["b"], P["f"], P["res"]
    t = int(np.argmin(np.abs(res.evals - P["sigma"])))
    E = res.evals[t]
    psi = res.evecs[:, t].contiguous()
    gap = float(np.min(np.abs(np.delete(res.evals, t) - E)))
    dE, dz2, z, info = gpu.eig_grad(b, f, E, psi, tol=1e-12)
    say(f"  L=20 adjoint: E={E:.12f} gap>={gap:.1e} minres={info.iters}")
    assert info.status == 0
    assert abs(dE.sum()) <= 1e-10 and abs(dz2.sum()) <= 1e-7 * max(1.0, np.abs(dz2).max())
    # Hellmann-Feynman against the oracle's expectation value of -S^z_j
    dE_ref = adjoint.hellmann_feynman(P["L"], psi.cpu().numpy())
    assert np.abs(dE - dE_ref).max() <= 1e-12
    delta = 1e-7
    for j in (0, 9, 16):
        Ep, z2p = [], []
        for sgn in (1.0, -1.0):
            hp = f.copy()
            hp[j] += sgn * delta
            v = _inverse_iteration(gpu, torch, b, hp, E, psi)
            Ep.append(float(torch.dot(v, gpu.apply_H(b, hp, 0.0, v))))
            z2p.append(abs(gpu.twist_expect(b, v)[0]) ** 2)
        dE_fd = (Ep[0] - Ep[1]) / (2 * delta)
        dz2_fd = (z2p[0] - z2p[1]) / (2 * delta)
        say(f"    site {j + 1}: dE={dE[j]:+.9f} fd={dE_fd:+.9f}  dz2={dz2[j]:+.6e} fd={dz2_fd:+.6e}")
        assert abs(dE[j] - dE_fd) <= 2e-5
        assert abs(dz2[j] - dz2_fd) <= 1e-3 * max(1.0, abs(dz2[j]))
