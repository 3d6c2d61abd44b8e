#!/usr/bin/env python3
"""Benchmark of the hot path on one MI355X.

Workload (default): the L=22 batch of the method's mixed-precision
experiment: 32 disorder realizations, h = 3.5, n = C(22, 11) = 705 432,
sigma at the spectral midpoint of each realization.

A timed step applies (H_r - sigma_r) to a resident FP64 vector for every
realization r of the batch (32 x 16n = 361 MB of algorithmic HBM traffic,
more than the 256 MB last-level cache). ``value`` is the algorithmic
apply_H bandwidth (16n bytes per product: read x once, write y once) of the
whole step; the roofline object reports the same figure against the HBM
peak. Time per MINRES iteration at L=22 (FP64 and FP32-inner) and, with
--eig, seconds per converged eigenpair at L=22 are reported beside it.

The CPU baseline is the oracle's sparse matrix-vector product on the host
cores over a bounded sample of the same workload.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--eig] [--no-cpu]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

HBM_PEAK_GBS = 8000.0
WORKLOAD = "mixed_L22"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--realizations", type=int, default=32)
    ap.add_argument("--eig", action="store_true", help="also time an L=22 eigensolve")
    ap.add_argument("--eig-nev", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--minres-iters", type=int, default=1000)
    ap.add_argument("--profile-run", action="store_true",
                    help="counter pass: 10 batched applies and 10 plain copies of the same size")
    return ap.parse_args()


def cpu_baseline(fields, sigmas, L, budget_s=15.0):
    """Oracle CSR product on the host, bounded to about budget_s seconds."""
    from oracle import model
    nthreads = 1   # scipy's CSR matvec runs on one thread
    t_build = time.perf_counter()
    H = model.hamiltonian_csr(L, fields[0])
    t_build = time.perf_counter() - t_build
    n = H.shape[0]
    x = np.random.default_rng(1).standard_normal(n)
    done = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < budget_s:
        y = H @ x - sigmas[0] * x
        done += 1
    dt = time.perf_counter() - t0
    del y
    return {
        "value": round(16.0 * n * done / dt / 1e9, 3), "unit": "GB/s", "cores": nthreads,
        "kind": "oracle",
        "sample": f"{done} products (H - sigma) x of realization 0 at L={L} with the oracle's "
                  f"scipy CSR matrix (build {t_build:.1f} s excluded), {dt:.1f} s",
    }


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
        sys.exit(2)
    import torch

    import paper_2203_09732_amd as mbl
    from workloads import WORKLOADS, disorder_fields

    cfg = WORKLOADS[WORKLOAD]
    L, hdis = cfg["L"], cfg["h"]
    R = args.realizations
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    from paper_2203_09732_amd import tune
    basis = mbl.Basis(L, tune.best_lo_bits(L, R, "fp64"))
    n = basis.n
    fields = [disorder_fields(L, hdis, s) for s in cfg["seeds"][:R]]
    sigmas = []
    for f in fields:
        if args.profile_run:       # the product's cost does not depend on the shift
            sigmas.append(0.0)
            continue
        _, _, sg = mbl.sigma_midpoint(basis, f, 1e-10)
        sigmas.append(sg)
    g = torch.Generator(device="cuda").manual_seed(1)
    # interleaved batch: element (i, r) at i * R + r
    g = torch.Generator(device="cuda").manual_seed(1)
    X = torch.randn((n, R), dtype=torch.float64, device=dev, generator=g)
    Y = torch.empty_like(X)
    batch = mbl.Batch(basis, R)
    stream = torch.cuda.current_stream()

    def step():
        mbl.apply_H_batched(basis, batch, fields, sigmas, X, Y)

    if args.profile_run:
        # reference for the byte counters: a plain device copy moving the same
        # algorithmic bytes (read 8nR, write 8nR) as one batched apply
        for _ in range(10):
            step()
        for _ in range(10):
            Y.copy_(X)
        torch.cuda.synchronize()
        print(json.dumps({"profile_run": True, "bytes_per_apply": 16 * n * R,
                          "bytes_per_copy": 16 * n * R}))
        return

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_s = e0.elapsed_time(e1) * 1e-3
    ms_per_step = gpu_s / args.steps * 1e3
    bytes_per_launch = 16.0 * n * R
    avg_launch = gpu_s / args.steps
    achieved = bytes_per_launch / avg_launch / 1e9
    value = achieved

    # the same products one realization per launch (single-realization kernel)
    xs = [X[:, r].contiguous() for r in range(R)]
    ys = [torch.empty_like(xs[0]) for _ in range(R)]
    for r in range(R):
        mbl.apply_H(basis, fields[r], sigmas[r], xs[r], ys[r])
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(max(1, args.steps // 10)):
        for r in range(R):
            mbl.apply_H(basis, fields[r], sigmas[r], xs[r], ys[r])
    e1.record(stream)
    torch.cuda.synchronize()
    single_s = e0.elapsed_time(e1) * 1e-3 / (max(1, args.steps // 10) * R)
    del xs, ys

    # MINRES iteration time at L=22: one realization (FP64, FP32-inner) and the
    # whole batch in lockstep (FP64, FP32-inner), fixed iteration counts
    ws = mbl.Workspace(basis, 0)
    minres = {}
    rhs = (X[:, 0] / X[:, 0].norm()).contiguous()
    for prec in ("fp64", "fp32_inner"):
        x = torch.zeros_like(rhs)
        torch.cuda.synchronize()
        t = time.perf_counter()
        _, info = mbl.minres_solve(basis, fields[0], sigmas[0], rhs, x, tol=1e-300,
                                   kmax=args.minres_iters, precision=prec, ws=ws)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        minres["single_" + prec] = {"iters": int(info.iters),
                                    "us_per_iter": round(dt / max(info.iters, 1) * 1e6, 2),
                                    "us_per_realization_iter": round(dt / max(info.iters, 1) * 1e6, 2)}
    Bn = (X / X.norm(dim=0, keepdim=True)).contiguous()
    for prec in ("fp64", "fp32_inner"):
        torch.cuda.synchronize()
        t = time.perf_counter()
        _, its, _, _ = mbl.minres_solve_batched(basis, batch, fields, sigmas, Bn, tol=1e-300,
                                               kmax=max(1, args.minres_iters // 10), precision=prec)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        it = int(its.max())
        minres["batched_" + prec] = {"iters": it, "realizations": R,
                                     "us_per_iter": round(dt / max(it, 1) * 1e6, 2),
                                     "us_per_realization_iter": round(dt / max(it, 1) / R * 1e6, 2)}

    out = {
        "metric": "apply_H HBM GB/s + sec per converged eigenpair at L=22, FP64 vs mixed/batched",
        "value": round(value, 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": WORKLOAD, "L": L, "n": n, "h": hdis, "realizations": R,
                   "lo_bits": basis.lo_bits,
                   "sigma": "spectral midpoint per realization",
                   "step": "one batched apply_H over all realizations (interleaved n x R)"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": f"k_bapply<double,0,false,{L},{basis.lo_bits}>",
                     "bytes_per_launch": bytes_per_launch, "avg_launch_us": round(avg_launch * 1e6, 3)},
        "apply_single_realization": {"GBps": round(16.0 * n / single_s / 1e9, 1),
                                     "avg_launch_us": round(single_s * 1e6, 3)},
        "minres_L22": minres,
        "wall_s": round(wall, 3),
    }
    if args.eig:
        from workloads import start_vector
        v0 = torch.as_tensor(start_vector(n, 0), device=dev)
        t = time.perf_counter()
        res = mbl.si_lanczos(basis, fields[0], sigmas[0], args.eig_nev, v0=v0)
        dt = time.perf_counter() - t
        out["sec_per_eigenpair_L22_fp64"] = {"value": round(dt / max(res.nconv, 1), 2), "nev": args.eig_nev,
                                             "nconv": res.nconv, "steps": res.steps,
                                             "minres_iters": res.minres_iters}
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(fields, sigmas, L)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
