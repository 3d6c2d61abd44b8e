"""Largest single-GPU workload: L = 26, n = 10 400 600 (h = 3.8, seed 0).

Full-size launches checked on sampled rows by the oracle's row-by-row
definition, device memory of a workspace linear in n (the MINRES vectors,
the Lanczos vectors and the basis), and bounded MINRES runs in both
precisions. A converged mid-spectrum eigenpair at this size needs of order
10^7 MINRES iterations per Lanczos step, far beyond a test."""
import sys

import numpy as np
import pytest

from oracle import model
from test_gpu_parity import dev, host, oracle_rows
from workloads import disorder_fields, gaussian_vector

pytestmark = pytest.mark.gpu

L26 = 26


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


@pytest.fixture(scope="module")
def states26():
    return model.sector_states(L26)


def test_L26_workspace_memory_linear_in_n(gpu, torch):
    """Workspace bytes = 8 n (13 vectors: z and d pairs, a ring of three q and
    p of MINRES,
    the FP32-inner correction, residual and scratch, Lanczos w and x; plus
    mmax + 1 Lanczos basis vectors) and O(1) scratch. With the caller's b
    and x, MINRES holds the paper's 9 vectors (its device memory model)."""
    b = gpu.Basis(L26)
    assert b.n == 10_400_600
    for mmax in (0, 70):
        ws = gpu.Workspace(b, mmax)
        model_bytes = 8 * b.n * (13 + (mmax + 1 if mmax > 0 else 0))
        say(f"L=26 mmax={mmax}: workspace {ws.bytes / 2**30:.3f} GiB, model {model_bytes / 2**30:.3f} GiB")
        assert 0 <= ws.bytes - model_bytes <= 16 << 20
        del ws


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_L26_apply_sampled_rows(gpu, torch, states26, precision):
    say(f"apply L=26 sampled rows {precision}")
    h = disorder_fields(L26, 3.8, 0)
    b = gpu.Basis(L26)
    x = gaussian_vector(b.n, 26)
    if precision == "fp32":
        x = x.astype(np.float32)
        y = host(gpu.apply_H(b, h, -0.3, dev(torch, x, torch.float32))).astype(np.float64)
        x = x.astype(np.float64)
        tol = 2e-6
    else:
        y = host(gpu.apply_H(b, h, -0.3, dev(torch, x)))
        tol = 1e-13
    rng = np.random.default_rng(26)
    rows = np.unique(np.concatenate([rng.integers(0, b.n, 3000), [0, 1, b.n - 2, b.n - 1]]))
    yref = oracle_rows(L26, h, -0.3, x, rows, states26)
    assert np.abs(y[rows] - yref).max() <= tol * np.abs(yref).max()


@pytest.mark.parametrize("precision", ["fp64", "fp32_inner"])
def test_L26_minres_bounded(gpu, torch, precision):
    """300 iterations at the spectral midpoint: the solver stops at kmax with
    a warning, a finite residual below its start, and x consistent with it."""
    say(f"minres L=26 kmax=300 {precision}")
    h = disorder_fields(L26, 3.8, 0)
    b = gpu.Basis(L26)
    _, _, sigma = gpu.sigma_midpoint(b, h, 1e-10)
    rhs = dev(torch, gaussian_vector(b.n, 27))
    rhs /= torch.linalg.norm(rhs)
    x, info = gpu.minres_solve(b, h, sigma, rhs, tol=1e-12, kmax=300, precision=precision)
    say(f"  status={info.status} iters={info.iters} phi={info.phi:.3e} true_res={info.true_res:.3e}")
    assert info.status == gpu.WARN_NOCONV
    assert info.iters >= 300 and np.isfinite(info.phi) and 0 < info.true_res < 1.0
    r = rhs - gpu.apply_H(b, h, sigma, x)
    assert abs(float(torch.linalg.norm(r)) - info.true_res) <= 1e-6 * max(info.true_res, 1e-12)
