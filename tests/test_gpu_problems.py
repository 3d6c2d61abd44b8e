"""Many realizations of uneven chain length in one call
(mbl_si_lanczos_problems): the persistent per-workgroup solver (L <= 16)
against the oracle's dense eigenpairs, the stored L = 16 sparse reference and
the single-realization path; the streaming batches the call runs for L >= 18
against the stored L = 18 sparse reference, in a call that mixes both, and at
small L (40 realizations on 32 lanes) against the dense eigenpairs.

Bars as for mbl_si_lanczos: sigma and the extremes 1e-10 relative; eigenvalues
|E - E_ref| / max(|E_ref|, 1) <= 1e-10; 1 - |<u, u_ref>| <= 1e-10; explicit
residual <= 1e-10 escale and equal to the oracle's recomputation; twist
|z - z_ref| <= 2 ||u - u_ref|| + 1e-12.
"""
import json
import os
import sys

import numpy as np
import pytest

from oracle import lanczos, model, twist
from workloads import disorder_fields

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _check_dense(L, f, r, nev, sigma=None):
    H = model.hamiltonian_dense(L, f)
    w = np.linalg.eigvalsh(H)
    escale = max(abs(w[0]), abs(w[-1]))
    if sigma is None:
        sigma = 0.5 * (w[0] + w[-1])
        assert abs(r.sigma - sigma) <= 1e-10 * escale, (r.sigma, sigma)
    else:
        assert r.sigma == sigma
    E, V = lanczos.eigenpairs_dense(H, r.sigma, nev)
    assert r.status == 0 and r.nconv == nev, (r.status, r.nconv)
    assert np.all(np.abs(r.evals - E) / np.maximum(np.abs(E), 1) <= 1e-10), r.evals - E
    U = r.evecs.cpu().numpy()
    ov = np.abs(np.sum(U * V, axis=0))
    assert np.all(1 - ov <= 1e-10), 1 - ov
    rr = lanczos.eigen_residuals(H, r.evals, U)
    assert np.all(rr <= 1e-10 * escale)
    assert np.allclose(r.resid, rr, rtol=1e-6, atol=1e-14)
    dpsi = np.minimum(np.linalg.norm(U - V, axis=0), np.linalg.norm(U + V, axis=0))
    assert np.all(np.abs(r.z - twist.twist_overlap(L, V)) <= 2 * dpsi + 1e-12)
    assert np.abs(r.z - twist.twist_overlap(L, U)).max() <= 1e-13


def test_mixed_lengths_against_dense_oracle(gpu):
    probs = []
    for k, (L, h, nev) in enumerate([(8, 3.0, 3), (10, 2.0, 4), (12, 3.0, 6), (14, 4.0, 5),
                                     (12, 1.0, 4), (10, 4.0, 2), (14, 3.0, 6), (12, 2.0, 3),
                                     (8, 1.0, 4), (14, 2.0, 4)]):
        probs.append(dict(L=L, h=disorder_fields(L, h, 100 + k), nev=nev))
    say(f"problems: {len(probs)} realizations, L = {sorted(set(p['L'] for p in probs))}")
    st, res = gpu.si_lanczos_problems(probs, seed=3, minres_kmax=400_000)
    assert st == 0
    for p, r in zip(probs, res):
        say(f"  L={r.L} nev={p['nev']} steps={r.steps} minres={r.minres_iters} "
            f"max_rel={r.max_rel_resid:.1e} t={r.seconds:.2f}s")
        _check_dense(p["L"], p["h"], r, p["nev"])


def test_given_shift_and_single_path_agree(gpu):
    import torch
    L, nev = 12, 4
    f = disorder_fields(L, 3.0, 77)
    sigma = 0.137
    st, res = gpu.si_lanczos_problems([dict(L=L, h=f, nev=nev, sigma=sigma)], seed=5,
                                      minres_kmax=400_000)
    assert st == 0
    _check_dense(L, f, res[0], nev, sigma=sigma)
    b = gpu.Basis(L)
    single = gpu.si_lanczos(b, f, sigma, nev, seed=5)
    assert np.all(np.abs(single.evals - res[0].evals) <= 1e-12 * np.maximum(1, np.abs(single.evals)))
    # the same seeded start vector (SplitMix64 of seed, index)
    assert res[0].steps == single.steps


def _check_stored(g, r):
    """A result against a stored sparse reference: eigenvalues, the oracle's
    CSR residual and the Davis-Kahan overlap bound with the stored gaps."""
    L, nev = g["L"], g["nev"]
    f = np.array(g["fields"])
    escale = max(abs(g["E_min"]), abs(g["E_max"]))
    say(f"  L={L} steps={r.steps} minres={r.minres_iters} sigma={r.sigma:.12f} t={r.seconds:.1f}s")
    assert r.status == 0 and r.nconv == nev
    assert abs(r.sigma - g["sigma"]) <= 1e-10 * escale
    Eref = np.array(g["evals"])
    assert np.all(np.abs(r.evals - Eref) / np.maximum(np.abs(Eref), 1) <= 1e-10)
    U = r.evecs.cpu().numpy()
    rr = lanczos.eigen_residuals(model.hamiltonian_csr(L, f), r.evals, U)
    assert np.all(rr <= 1e-10 * escale)
    assert np.allclose(r.resid, rr, rtol=1e-6, atol=1e-14)
    spec = np.array(g["window"])
    delta = np.array([np.min(np.abs(np.delete(spec, np.argmin(np.abs(spec - e))) - e))
                      for e in r.evals])
    deficit = 1 - np.sqrt(1 - np.minimum(1.0, rr / delta) ** 2)
    assert np.all(deficit <= 1e-10)
    zref = np.array(g["z_re"]) + 1j * np.array(g["z_im"])
    assert np.all(np.abs(r.z - zref) <= 2 * np.sqrt(2 * deficit) + 1e-12)
    assert np.abs(r.z - twist.twist_overlap(L, U)).max() <= 1e-13


def test_L16_against_stored_sparse_reference(gpu):
    g = json.load(open(os.path.join(HERE, "golden", "si_L16_h3_seed0.json")))
    L, nev = g["L"], g["nev"]
    f = np.array(g["fields"])
    escale = max(abs(g["E_min"]), abs(g["E_max"]))
    probs = [dict(L=L, h=f, nev=nev, sigma=g["sigma"], escale=escale), dict(L=L, h=f, nev=nev)]
    st, res = gpu.si_lanczos_problems(probs, seed=9, minres_kmax=400_000)
    assert st == 0
    for r in res:
        _check_stored(g, r)


def test_L18_streaming_route_in_a_mixed_call(gpu):
    """L = 18 (stored reference, sigma computed by the call) beside an L = 12
    realization of the persistent launch and a second L = 18 realization of
    other fields that shares the streaming batch."""
    g = json.load(open(os.path.join(HERE, "golden", "si_L18_h3_seed0.json")))
    f = np.array(g["fields"])
    probs = [dict(L=12, h=disorder_fields(12, 3.0, 41), nev=4),
             dict(L=18, h=f, nev=g["nev"]),
             dict(L=18, h=disorder_fields(18, 4.0, 42), nev=2)]
    st, res = gpu.si_lanczos_problems(probs, seed=13, minres_kmax=2_000_000)
    assert st == 0
    _check_dense(12, probs[0]["h"], res[0], 4)
    _check_stored(g, res[1])
    r = res[2]
    assert r.status == 0 and r.nconv == 2 and r.L == 18
    H = model.hamiltonian_csr(18, probs[2]["h"])
    rr = lanczos.eigen_residuals(H, r.evals, r.evecs.cpu().numpy())
    lo, hi = lanczos.extremal_eigenvalues(H)
    escale = max(abs(lo), abs(hi))
    assert abs(r.sigma - 0.5 * (lo + hi)) <= 1e-10 * escale
    assert np.all(rr <= 1e-10 * escale)


def test_streaming_lanes_take_new_realizations(gpu, monkeypatch):
    """The streaming batched form at small L (MBL_PERSISTENT_MAX_L=10 sends
    L = 12 and 14 there): 40 realizations of L = 12 on 32 lanes (8 lanes take
    a second realization when their first has converged) and 3 of L = 14 with
    another nev, each against the oracle's dense eigenpairs."""
    monkeypatch.setenv("MBL_PERSISTENT_MAX_L", "10")
    probs = []
    for k in range(40):
        probs.append(dict(L=12, h=disorder_fields(12, (1.0, 2.0, 3.0, 4.0)[k % 4], 300 + k),
                          nev=4 if k % 3 else 6))
    for k in range(3):
        probs.append(dict(L=14, h=disorder_fields(14, 3.0, 400 + k), nev=5))
    st, res = gpu.si_lanczos_problems(probs, seed=21, minres_kmax=400_000)
    assert st == 0
    for p, r in zip(probs, res):
        _check_dense(p["L"], p["h"], r, p["nev"])
    say(f"  streaming: {len(res)} realizations, steps {min(r.steps for r in res)}..."
        f"{max(r.steps for r in res)}, t={res[0].seconds:.1f}s")


def test_problem_array_rejects_bad_arguments(gpu):
    for bad in (dict(L=11, h=np.zeros(11), nev=2), dict(L=10, h=np.zeros(10), nev=0),
                dict(L=10, h=np.zeros(10), nev=33), dict(L=10, h=np.full(10, np.nan), nev=2),
                dict(L=10, h=np.zeros(10), nev=2, sigma=np.inf)):
        with pytest.raises(gpu.MblError) as e:
            gpu.si_lanczos_problems([bad])
        assert e.value.status == gpu.ERR_ARG
    with pytest.raises(gpu.MblError):
        gpu.si_lanczos_problems([dict(L=10, h=np.zeros(10), nev=2)], minres_tol=0.0)
