"""Parity of the batched (interleaved, lockstep) HIP path against the CPU
oracle and against the single-realization path, through the C ABI."""
import math
import sys

import numpy as np
import pytest

from oracle import lanczos, minres, model, twist
from workloads import disorder_fields, gaussian_vector, start_vector

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


def _batch_inputs(L, R, h=3.0, seed0=0):
    fields = [disorder_fields(L, h, seed0 + r) for r in range(R)]
    sig = [0.1 * r - 0.3 for r in range(R)]
    return fields, sig


@pytest.mark.parametrize("L,R", [(12, 2), (12, 8), (14, 32), (16, 4), (16, 16), (16, 32)])
def test_apply_batched_dense_parity(gpu, torch, L, R):
    say(f"apply batched L={L} R={R}")
    b = gpu.Basis(L)
    bt = gpu.Batch(b, R)
    fields, sig = _batch_inputs(L, R)
    X = np.stack([gaussian_vector(b.n, 50 + r) for r in range(R)], axis=1)
    Y = gpu.apply_H_batched(b, bt, fields, sig, torch.as_tensor(X, device="cuda")).cpu().numpy()
    for r in range(R):
        H = model.hamiltonian_csr(L, fields[r])
        yref = H @ X[:, r] - sig[r] * X[:, r]
        assert np.abs(Y[:, r] - yref).max() <= 1e-13 * np.abs(yref).max()
    # the single-realization kernel sums in the same order
    ys = gpu.apply_H(b, fields[R - 1], sig[R - 1], torch.as_tensor(np.ascontiguousarray(X[:, R - 1]), device="cuda"))
    assert np.abs(ys.cpu().numpy() - Y[:, R - 1]).max() <= 1e-15 * np.abs(Y[:, R - 1]).max()


def test_apply_batched_f32(gpu, torch):
    say("apply batched f32 L=14 R=8")
    L, R = 14, 8
    b = gpu.Basis(L)
    bt = gpu.Batch(b, R)
    fields, sig = _batch_inputs(L, R)
    X = np.stack([gaussian_vector(b.n, 70 + r) for r in range(R)], axis=1).astype(np.float32)
    Y = gpu.apply_H_batched(b, bt, fields, sig, torch.as_tensor(X, device="cuda")).cpu().numpy()
    for r in range(R):
        yref = model.hamiltonian_csr(L, fields[r]) @ X[:, r].astype(np.float64) - sig[r] * X[:, r]
        assert np.abs(Y[:, r] - yref).max() <= 2e-6 * np.abs(yref).max()


@pytest.mark.parametrize("L,R,split", [(22, 32, "tuned"), (22, 32, "default"), (22, 32, "staged"),
                                       (24, 8, "default")])
def test_apply_batched_sampled_rows_large(gpu, torch, L, R, split):
    """Full-size batched launches, rows checked one by one by the oracle; the
    tuned split at L=22, R=32 is the launch the benchmark times (with the
    bench's fields: h = 3.5, seeds 0..31); split 10 at R = 32 takes the
    block-staged product."""
    from paper_2203_09732_amd import tune
    lo = {"tuned": tune.best_lo_bits(L, R, "fp64"), "staged": 10}.get(split, 0)
    say(f"apply batched sampled L={L} R={R} lo_bits={lo or 'default'}")
    b = gpu.Basis(L, lo)
    bt = gpu.Batch(b, R)
    if split == "tuned":
        fields, sig = [disorder_fields(L, 3.5, s) for s in range(R)], [-0.1] * R
    else:
        fields, sig = _batch_inputs(L, R, h=3.5)
    g = torch.Generator(device="cuda").manual_seed(3)
    X = torch.randn((b.n, R), dtype=torch.float64, device="cuda", generator=g)
    Y = gpu.apply_H_batched(b, bt, fields, sig, X).cpu().numpy()
    Xh = X.cpu().numpy()
    states = model.sector_states(L)
    rng = np.random.default_rng(L)
    rows = np.unique(np.concatenate([rng.integers(0, b.n, 1500), [0, b.n - 1]]))
    for r in (0, R // 2, R - 1):
        st = states[rows]
        yref = (model.diagonal(L, fields[r], st) - sig[r]) * Xh[rows, r]
        for (a, c) in model.bonds(L):
            anti = ((st >> (a - 1)) & 1) != ((st >> (c - 1)) & 1)
            fl = st ^ ((1 << (a - 1)) | (1 << (c - 1)))
            idx = np.clip(np.searchsorted(states, fl), 0, len(states) - 1)
            yref = yref + np.where(anti, 0.5 * Xh[idx, r], 0.0)
        assert np.abs(Y[rows, r] - yref).max() <= 1e-13 * np.abs(yref).max()


def _problems(L, R, h=3.0, seed0=0):
    fields, Hs, sig = [], [], []
    for r in range(R):
        f = disorder_fields(L, h, seed0 + r)
        H = model.hamiltonian_csr(L, f)
        w = np.linalg.eigvalsh(H.toarray())
        fields.append(f)
        Hs.append(H)
        sig.append(0.5 * (w[0] + w[-1]))
    return fields, Hs, sig


@pytest.mark.parametrize("precision", ["fp64", "fp32_inner"])
def test_minres_batched_parity(gpu, torch, precision):
    say(f"minres batched L=12 R=4 {precision}")
    L, R = 12, 4
    fields, Hs, sig = _problems(L, R)
    b = gpu.Basis(L)
    bt = gpu.Batch(b, R)
    B = np.stack([gaussian_vector(b.n, 90 + r) for r in range(R)], axis=1)
    B /= np.linalg.norm(B, axis=0)
    x, its, phi, st = gpu.minres_solve_batched(b, bt, fields, sig, torch.as_tensor(B, device="cuda"),
                                               tol=1e-12, precision=precision)
    assert st == 0 and np.all(phi < 1e-12)
    X = x.cpu().numpy()
    for r in range(R):
        xd = minres.solve_dense(Hs[r].toarray(), sig[r], B[:, r])
        assert np.linalg.norm(X[:, r] - xd) / np.linalg.norm(xd) <= 1e-8
    if precision == "fp64":
        # same iteration count as the single-realization solver (same recurrence)
        xs, info = gpu.minres_solve(b, fields[1], sig[1], torch.as_tensor(np.ascontiguousarray(B[:, 1]), device="cuda"), tol=1e-12)
        assert abs(info.iters - its[1]) <= 0.05 * its[1] + 5


def test_schedule_knobs_keep_results(gpu, torch):
    """The launch schedule (mbl_batch_set_schedule) changes how the work is
    launched, not what is computed: the graph length and the d/x pass length
    keep the batched MINRES bit for bit (same kernels, same per-element
    arithmetic); another grid reorders the partial sums only (rounding); the
    apply has no sums and stays bit for bit. Bad values are MBL_ERR_ARG."""
    say("batched schedule knobs L=14 R=8")
    L, R = 14, 8
    fields, Hs, sig = _problems(L, R, seed0=30)
    b = gpu.Basis(L)
    bt = gpu.Batch(b, R)
    B = np.stack([gaussian_vector(b.n, 130 + r) for r in range(R)], axis=1)
    B /= np.linalg.norm(B, axis=0)
    Bt = torch.as_tensor(B, device="cuda")
    x0, its0, phi0, st = gpu.minres_solve_batched(b, bt, fields, sig, Bt, tol=1e-12)
    assert st == 0
    y0 = gpu.apply_H_batched(b, bt, fields, sig, Bt)
    for grid, gi, dx in [(0, 8, 1), (0, 32, 2), (0, 16, 4), (128, 16, 4), (64, 8, 2), (512, 32, 1)]:
        bt.set_schedule(grid, gi, dx)
        x, its, phi, st = gpu.minres_solve_batched(b, bt, fields, sig, Bt, tol=1e-12)
        y = gpu.apply_H_batched(b, bt, fields, sig, Bt)
        say(f"  grid={grid} graph={gi} dx={dx}: iterations {list(its)}")
        assert st == 0 and torch.equal(y, y0)
        if grid == 0:
            assert torch.equal(x, x0) and np.array_equal(its, its0)
        else:
            # the MINRES bar against a dense solve; the count at the threshold
            # moves with rounding as the oracle's own does (up to ~7 %)
            assert (torch.linalg.norm(x - x0) / torch.linalg.norm(x0)).item() <= 1e-8
            assert np.all(np.abs(its - its0) <= 0.1 * its0 + 5)
    for bad in [(7, 0, 0), (1024, 0, 0), (0, 12, 0), (0, 0, 3)]:
        with pytest.raises(gpu.MblError) as e:
            bt.set_schedule(*bad)
        assert e.value.status == gpu.ERR_ARG


@pytest.mark.parametrize("precision", ["fp64", "fp32_inner"])
def test_si_lanczos_batched_parity(gpu, torch, precision):
    say(f"si_lanczos batched L=12 R=4 nev=4 {precision}")
    L, R, nev = 12, 4, 4
    fields, Hs, sig = _problems(L, R, seed0=10)
    b = gpu.Basis(L)
    bt = gpu.Batch(b, R, mmax=60, nevmax=nev)
    V0 = np.stack([start_vector(b.n, r) for r in range(R)], axis=1)
    res = gpu.si_lanczos_batched(b, bt, fields, sig, nev, v0=torch.as_tensor(V0, device="cuda"),
                                 precision=precision)
    say(f"  steps={res.steps} nconv={res.nconv} minres={res.minres_iters} t={res.seconds:.2f}s")
    assert res.status == 0 and np.all(res.nconv == nev)
    U = res.evecs.cpu().numpy()
    z = gpu.twist_expect_batched(b, bt, res.evecs)
    for r in range(R):
        E, Vr = lanczos.eigenpairs_dense(Hs[r].toarray(), sig[r], nev)
        assert np.all(np.abs(res.evals[r] - E) / np.maximum(np.abs(E), 1) <= 1e-10)
        Ur = U[:, :, r].T
        ov = np.abs(np.sum(Ur * Vr, axis=0))
        assert np.all(1 - ov <= 1e-10)
        dpsi = np.minimum(np.linalg.norm(Ur - Vr, axis=0), np.linalg.norm(Ur + Vr, axis=0))
        zr = twist.twist_overlap(L, Vr)
        assert np.all(np.abs(z[r] - zr) <= 2 * dpsi + 1e-12)
        rr = lanczos.eigen_residuals(Hs[r], res.evals[r], Ur)
        assert np.allclose(res.resid[r], rr, rtol=1e-6, atol=1e-14)


def test_si_lanczos_batched_frozen_realization_with_poisoned_memory(gpu, torch):
    """Realizations that converge early are frozen with zero coefficients
    while the others go on; their later Lanczos columns are never computed.
    Device memory filled with NaN and released just before the batch is
    created must not reach any result (a zero coefficient reads nothing)."""
    say("si_lanczos batched frozen realization, NaN-poisoned memory")
    L, R, nev = 12, 2, 2
    fields = [disorder_fields(L, 2.0, 100), disorder_fields(L, 4.0, 102)]
    b = gpu.Basis(L)
    sig = [gpu.sigma_midpoint(b, f, 1e-12)[2] for f in fields]
    junk = torch.full((64 << 20,), float("nan"), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    del junk
    torch.cuda.empty_cache()
    bt = gpu.Batch(b, R, mmax=46, nevmax=nev)
    res = gpu.si_lanczos_batched(b, bt, fields, sig, nev, mmax=46, escale=[15.0, 15.0], seed=1234)
    assert res.status == 0 and np.all(res.nconv == nev)
    assert res.steps[0] != res.steps[1]   # one realization was frozen while the other ran
    for r in range(R):
        H = model.hamiltonian_dense(L, fields[r])
        E, _ = lanczos.eigenpairs_dense(H, sig[r], nev)
        assert np.all(np.abs(res.evals[r] - E) / np.maximum(np.abs(E), 1) <= 1e-10)


def test_staged_product_matches_row_product(gpu, torch):
    """The block-staged product (split 10, R = 32) against the row product at
    another split, on the same full-size L = 22 input: the same terms summed
    in another order, so equal to rounding."""
    L, R = 22, 32
    fields, sig = _batch_inputs(L, R, h=3.5)
    out = {}
    for lo in (10, 11):
        b = gpu.Basis(L, lo)
        bt = gpu.Batch(b, R)
        X = torch.randn((b.n, R), dtype=torch.float64, device="cuda",
                        generator=torch.Generator(device="cuda").manual_seed(5))
        out[lo] = gpu.apply_H_batched(b, bt, fields, sig, X)
    d = (out[10] - out[11]).abs().max().item()
    say(f"  staged vs row product: max |dy| = {d:.2e}")
    assert d <= 1e-14 * out[11].abs().max().item()


def test_staged_minres_product(gpu, torch):
    """Batched MINRES at L = 14, R = 32 (split 10: the block-staged product
    with the Givens prologue and partial sums) against dense solves, and
    against the row product at split 7 on the same right-hand sides (the same
    recurrence with sums in another order). The iteration counts are printed,
    not compared: at tol 1e-12 the count at the threshold moves with rounding
    (by up to 25 % between these two runs), while the solutions agree."""
    L, R = 14, 32
    fields = [disorder_fields(L, 3.0, 60 + r) for r in range(R)]
    sig = [0.03 * r - 0.5 for r in range(R)]
    n = len(model.sector_states(L))
    B = np.stack([gaussian_vector(n, 160 + r) for r in range(R)], axis=1)
    B /= np.linalg.norm(B, axis=0)
    out = {}
    for lo in (10, 7):
        b = gpu.Basis(L, lo)
        bt = gpu.Batch(b, R)
        x, its, phi, st = gpu.minres_solve_batched(b, bt, fields, sig,
                                                   torch.as_tensor(B, device="cuda"), tol=1e-12)
        assert st == 0 and np.all(phi < 1e-12)
        out[lo] = (x.cpu().numpy(), its)
    X10, its10 = out[10]
    X7, its7 = out[7]
    say(f"  staged iterations {list(its10[:6])}..., row product {list(its7[:6])}...")
    for r in (0, 13, 31):
        xd = minres.solve_dense(model.hamiltonian_dense(L, fields[r]), sig[r], B[:, r])
        assert np.linalg.norm(X10[:, r] - xd) / np.linalg.norm(xd) <= 1e-8
    assert np.max(np.linalg.norm(X10 - X7, axis=0) / np.linalg.norm(X7, axis=0)) <= 1e-8
