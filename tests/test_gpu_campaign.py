"""Uneven-L campaign driver and graph-captured batched MINRES."""
import json
import os
import sys

import numpy as np
import pytest

from oracle import lanczos, model, twist
from workloads import batched_realization, disorder_fields, gaussian_vector

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


@pytest.mark.parametrize("mode", ["persistent", "lockstep"])
def test_campaign_uneven_lengths_and_resume(gpu, torch, tmp_path, mode):
    from paper_2203_09732_amd import campaign
    tasks = []
    for i in range(6):
        L = 12 if i % 2 == 0 else 14
        h = [2.0, 3.0, 4.0][i % 3]
        tasks.append(campaign.Task(i, L, h, disorder_fields(L, h, 100 + i)))
    path = str(tmp_path / "res.jsonl")
    say(f"campaign ({mode}) L in {{12, 14}}, 6 realizations, nev=2")
    recs = campaign.run(tasks, nev=2, results_path=path, log=say, mode=mode)
    assert len(recs) == 6
    for rec in recs:
        t = tasks[rec["index"]]
        H = model.hamiltonian_dense(t.L, t.fields)
        w = np.linalg.eigvalsh(H)
        sg = 0.5 * (w[0] + w[-1])
        assert abs(rec["sigma"] - sg) <= 1e-9 * max(abs(w[0]), abs(w[-1]))
        E, V = lanczos.eigenpairs_dense(H, rec["sigma"], 2)
        assert np.allclose(rec["evals"], E, atol=1e-10 * max(1, np.abs(E).max()))
        assert rec["nconv"] == 2
        z = np.array(rec["z_re"]) + 1j * np.array(rec["z_im"])
        zr = twist.twist_overlap(t.L, V)
        assert np.abs(z - zr).max() <= 1e-6
    # a second run finds every realization in the results file and does nothing
    again = campaign.run(tasks, nev=2, results_path=path, log=None, mode=mode)
    assert again == []
    assert len(open(path).read().strip().splitlines()) == 6


@pytest.mark.parametrize("R", [8, 32])
def test_batched_minres_graph_replays_match_eager(gpu, torch, R):
    """Several solves with graph replays, with eager work and syncs between
    them; each must equal the eager-launch result bit for bit (R = 32 at
    L = 14 runs the block-staged MINRES product)."""
    L = 14
    b = gpu.Basis(L)
    fields = [disorder_fields(L, 3.0, 200 + r) for r in range(R)]
    sig = [0.05 * r - 0.2 for r in range(R)]
    os.environ["MBL_BATCH_GRAPHS"] = "0"
    eager_bt = gpu.Batch(b, R)
    os.environ["MBL_BATCH_GRAPHS"] = "1"
    graph_bt = gpu.Batch(b, R)
    del os.environ["MBL_BATCH_GRAPHS"]
    for trial in range(3):
        say(f"graph replay trial {trial}")
        B = np.stack([gaussian_vector(b.n, 300 + 10 * trial + r) for r in range(R)], axis=1)
        Bt = torch.as_tensor(B / np.linalg.norm(B, axis=0), device="cuda")
        xe, ie, pe, _ = gpu.minres_solve_batched(b, eager_bt, fields, sig, Bt, tol=1e-10)
        # unrelated eager work between the replays
        gpu.apply_H_batched(b, graph_bt, fields, sig, Bt)
        torch.cuda.synchronize()
        xg, ig, pg, _ = gpu.minres_solve_batched(b, graph_bt, fields, sig, Bt, tol=1e-10)
        assert np.array_equal(ie, ig)
        assert torch.equal(xe, xg)


def test_campaign_mixed_sizes_sample_vs_oracle(gpu, torch):
    """Realizations of the mixed-size workload (chain length and disorder
    strength drawn per realization, seeded) with L in {14, 16}: sigma equals
    the oracle's midpoint, the nev = 6 eigenvalues nearest it equal the
    oracle's (dense at L = 14, sparse shift-invert at L = 16), and each z is
    within the bound 2 ||delta psi|| <= 2 resid / gap of the oracle's."""
    from paper_2203_09732_amd import campaign
    from workloads import batched_realizations
    reals = [r for r in batched_realizations(40) if r.L in (14, 16)][:10]
    assert {r.L for r in reals} == {14, 16}
    tasks = [campaign.Task(r.index, r.L, r.h, r.fields) for r in reals]
    say(f"campaign sample of the mixed-size workload: {[(r.index, r.L, r.h) for r in reals]}")
    recs = campaign.run(tasks, nev=6, log=say)
    assert len(recs) == len(reals)
    for rec in recs:
        r = next(x for x in reals if x.index == rec["index"])
        H = model.hamiltonian_csr(r.L, r.fields)
        lo, hi = lanczos.extremal_eigenvalues(H)
        assert abs(rec["sigma"] - 0.5 * (lo + hi)) <= 1e-9 * max(abs(lo), abs(hi))
        if r.L == 14:
            E, V = lanczos.eigenpairs_dense(H.toarray(), rec["sigma"], 6)
            w = np.linalg.eigvalsh(H.toarray())
        else:
            E, V = lanczos.eigenpairs_shift_invert_sparse(H, rec["sigma"], 10)
            keep = np.sort(np.argsort(np.abs(E - rec["sigma"]))[:6])
            w, E, V = E, E[keep], V[:, keep]
        assert rec["nconv"] == 6
        assert np.all(np.abs(np.array(rec["evals"]) - E) / np.maximum(np.abs(E), 1) <= 1e-10)
        gaps = np.array([np.min(np.abs(np.delete(w, np.argmin(np.abs(w - e))) - e)) for e in E])
        z = np.array(rec["z_re"]) + 1j * np.array(rec["z_im"])
        zr = twist.twist_overlap(r.L, V)
        bound = 2 * np.array(rec["resid"]) / gaps + 1e-9
        assert np.all(np.abs(z - zr) <= bound), (np.abs(z - zr), bound)
