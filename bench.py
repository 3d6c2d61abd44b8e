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
peak. Time per MINRES iteration at L=22 (FP64 and FP32-inner) and seconds
per converged eigenpair are reported beside it: measured at L=18 (the
largest chain whose eigen-runs fit the bench's few minutes; one FP64 pair at
L=22 takes about three minutes) in the single, batched and
FP32-inner forms, and at L=14 (the plain 10-pair workload) for comparison
with the oracle's dense solver on the host.

The CPU baseline is the oracle on the host cores over bounded samples: its
sparse matrix-vector product at L=22 (the headline unit), and seconds per
eigenpair of its dense eigensolver on the L=14 workload.

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
NPAIRS = 4          # distinct (x, y) pairs the timed applies rotate over
COUNTERS = os.path.join(ROOT, "profiles", "bapply_L22_R32_counters.md")


# the sources the batched apply kernel is compiled from
KERNEL_SOURCES = ["paper_2203_09732_amd/csrc/batched.hip", "paper_2203_09732_amd/csrc/brows.h",
                  "paper_2203_09732_amd/csrc/rows.h", "paper_2203_09732_amd/csrc/mbl_internal.h",
                  "include/mbl.h"]


def kernel_source_hash() -> str:
    """sha256 over the batched apply kernel's sources (file name, then content,
    in the order of KERNEL_SOURCES)."""
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        h.update(os.path.basename(rel).encode())
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def headline_kernel(L: int, lo_bits: int, R: int) -> str:
    """The kernel the library launches for the FP64 batched product: the
    block-staged one for split 10 at R = 32 (L = 14, 16, 22), else the row
    product of the split."""
    if lo_bits == 10 and R == 32 and L in (14, 16, 22):
        return f"k_bapply_staged<{L},0>"
    return f"k_bapply<double,0,false,{L},{lo_bits}>"


def measured_traffic(kernel: str):
    """HBM bytes per launch from the committed counter summary, or None when
    the kernel sources or the kernel instance differ from the ones counted."""
    try:
        fields = dict(line.split(": ", 1) for line in open(COUNTERS).read().splitlines()
                      if ": " in line and line.split(": ", 1)[0] in
                      ("source_sha256", "kernel", "traffic_bytes_per_launch"))
    except OSError:
        return None
    if fields.get("source_sha256", "").strip() != kernel_source_hash():
        return None
    if fields.get("kernel", "").strip() != kernel:
        return None
    return int(fields["traffic_bytes_per_launch"])


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--realizations", type=int, default=32)
    ap.add_argument("--eig-L", type=int, default=18, help="chain length of the eigenpair leg")
    ap.add_argument("--eig-nev", type=int, default=6)
    ap.add_argument("--eig-R", type=int, default=8, help="realizations of the batched eigen leg")
    ap.add_argument("--no-eig", action="store_true", help="skip the eigenpair leg")
    ap.add_argument("--eig-batched-mixed", action="store_true",
                    help="also time the lockstep FP32-inner eigen leg (minutes)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--largest", action="store_true",
                    help="also measure the L=26 workload (memory, apply, MINRES per iteration)")
    ap.add_argument("--minres-iters", type=int, default=1000)
    ap.add_argument("--profile-run", action="store_true",
                    help="counter pass: 10 batched applies and 10 plain copies of the same size")
    return ap.parse_args()


def host_info():
    """Host cores, CPU model and the BLAS the oracle's dense solver runs on."""
    info = {"nproc": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity")
            else os.cpu_count()}
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    info["cpu_model"] = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        import threadpoolctl
        blas = [p for p in threadpoolctl.threadpool_info() if p.get("user_api") == "blas"]
        if blas:
            info["blas"] = f"{blas[0].get('internal_api')} {blas[0].get('version')}"
            info["blas_threads"] = blas[0].get("num_threads")
    except Exception:
        pass
    return info


def cpu_baseline(fields, sigmas, L, budget_s=12.0):
    """The oracle on the host over bounded samples: its CSR product (H - sigma) x
    at the headline L (one thread: scipy's CSR product is serial), and seconds
    per eigenpair of its dense eigensolver (LAPACK through the threaded BLAS)
    on the L=14 workload (10 pairs nearest the spectral midpoint)."""
    from oracle import lanczos, model
    from workloads import WORKLOADS
    nthreads = 1
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
    del y, H
    info = host_info()
    cfg = WORKLOADS["plain_L14"]
    from workloads import disorder_fields
    Hd = model.hamiltonian_dense(cfg["L"], disorder_fields(cfg["L"], cfg["h"], cfg["seeds"][0]))
    t1 = time.perf_counter()
    w = np.linalg.eigvalsh(Hd)
    sigma14 = 0.5 * (w[0] + w[-1])
    E, _V = lanczos.eigenpairs_dense(Hd, sigma14, cfg["nev"])
    t_eig = time.perf_counter() - t1
    return {
        "value": round(16.0 * n * done / dt / 1e9, 3), "unit": "GB/s", "cores": nthreads,
        "kind": "oracle",
        "sample": f"{done} products (H - sigma) x of realization 0 at L={L} with the oracle's "
                  f"scipy CSR matrix (build {t_build:.1f} s excluded), {dt:.1f} s",
        "host": info,
        "sec_per_eigenpair_L14": {
            "value": round(t_eig / cfg["nev"], 4), "unit": "s per eigenpair",
            "threads": info.get("blas_threads"),
            "sample": f"oracle dense eigensolver (eigvalsh for sigma, then eigh and the "
                      f"{cfg['nev']} pairs nearest sigma) on the L={cfg['L']} h={cfg['h']} "
                      f"seed {cfg['seeds'][0]} workload, n={Hd.shape[0]}, {t_eig:.1f} s"},
    }


def progress(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def eig_leg(mbl, torch, L, nev, R, batched_mixed=False):
    """Seconds per converged eigenpair (explicit FP64 residual <= 1e-10 escale)
    of the whole path (sigma, SI-Lanczos with MINRES, Ritz vectors, residual
    checks, twist) at chain length L: one realization per call in FP64 and
    with FP32-inner MINRES, R realizations in lockstep in FP64 (the lockstep
    FP32-inner run only with batched_mixed), and the same R realizations in
    one problem-array call. Every call is timed whole, with sigma; nothing is
    projected."""
    from workloads import disorder_fields
    from paper_2203_09732_amd import tune
    h = 3.0
    fields = [disorder_fields(L, h, 5000 + r) for r in range(R)]
    out = {"L": L, "nev": nev, "h": h, "eig_tol": 1e-10, "minres_tol": 1e-12,
           "seeds": f"5000..{5000 + R - 1}"}
    for prec in ("fp64", "fp32_inner"):
        b = mbl.Basis(L)
        torch.cuda.synchronize()
        t = time.perf_counter()
        lo, hi, sg = mbl.sigma_midpoint(b, fields[0], 1e-12)
        res = mbl.si_lanczos(b, fields[0], sg, nev, escale=max(abs(lo), abs(hi)), seed=7,
                             precision=prec)
        mbl.twist_expect(b, res.evecs)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        progress(f"eig leg L={L} single {prec}: {dt:.1f} s, {res.nconv} pairs")
        out["single_" + prec] = {"value": round(dt / max(res.nconv, 1), 4), "nconv": int(res.nconv),
                                 "realizations": 1, "seconds": round(dt, 3), "steps": int(res.steps),
                                 "minres_iters": int(res.minres_iters),
                                 "max_rel_resid": float(res.max_rel_resid)}
        if prec == "fp64":
            # adjoint derivatives dE/dh and d|z|^2/dh of every converged pair
            torch.cuda.synchronize()
            t = time.perf_counter()
            its = 0
            for k in range(res.nconv):
                _, _, _, ginfo = mbl.eig_grad(b, fields[0], res.evals[k],
                                             res.evecs[:, k].contiguous(), tol=1e-12)
                its += ginfo.iters
            torch.cuda.synchronize()
            dt = time.perf_counter() - t
            progress(f"eig leg L={L} adjoint: {dt / max(res.nconv, 1):.2f} s per pair")
            out["adjoint_fp64"] = {"value": round(dt / max(res.nconv, 1), 4),
                                   "unit": "s per eigenpair (all L derivatives of E and |z|^2)",
                                   "minres_iters_per_pair": its // max(res.nconv, 1)}
            # eigenstate observables of the same pairs: half-chain entropy, spacing ratio
            torch.cuda.synchronize()
            t = time.perf_counter()
            S = mbl.entanglement_entropy(b, res.evecs)
            dt = time.perf_counter() - t
            out["observables_fp64"] = {"S_half_chain_mean": round(float(np.mean(S)), 6),
                                       "entropy_ms_per_vector": round(dt / len(S) * 1e3, 3),
                                       "r_mean": round(mbl.spacing_ratio(res.evals)[0], 6)}
        if prec != "fp64" and not batched_mixed:
            continue
        tp = "fp64" if prec == "fp64" else "fp32"
        bb = mbl.Basis(L, tune.best_lo_bits(L, R, tp))
        mmax = min(bb.n, 3 * nev + 40)
        bt = mbl.Batch(bb, R, mmax=mmax, nevmax=nev)
        tune.apply_schedule(bt, L, R, tp)
        torch.cuda.synchronize()
        t = time.perf_counter()
        sig, esc = [], []
        for f in fields:
            lo, hi, sg = mbl.sigma_midpoint(bb, f, 1e-12)
            sig.append(sg)
            esc.append(max(abs(lo), abs(hi)))
        resb = mbl.si_lanczos_batched(bb, bt, fields, sig, nev, mmax=mmax, escale=esc, seed=7,
                                      precision=prec)
        mbl.twist_expect_batched(bb, bt, resb.evecs)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        nconv = int(resb.nconv.sum())
        progress(f"eig leg L={L} batched R={R} {prec}: {dt:.1f} s, {nconv} pairs")
        out["batched_" + prec] = {"value": round(dt / max(nconv, 1), 4), "nconv": nconv,
                                  "realizations": R, "seconds": round(dt, 3),
                                  "steps_max": int(resb.steps.max()),
                                  "minres_iters": int(resb.minres_iters)}
    # the same R realizations through the problem-array call: the persistent
    # launch (L <= 16) or the streaming lanes (L >= 18), sigma included
    torch.cuda.synchronize()
    t = time.perf_counter()
    st, resp = mbl.si_lanczos_problems([dict(L=L, h=f, nev=nev) for f in fields], seed=7)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    nconv = int(sum(r.nconv for r in resp))
    progress(f"eig leg L={L} problem array ({R} realizations): {dt:.1f} s, {nconv} pairs")
    out["problems_fp64"] = {"value": round(dt / max(nconv, 1), 4), "nconv": nconv,
                            "realizations": R, "seconds": round(dt, 3),
                            "form": "persistent" if L <= 16 else "streaming",
                            "steps_max": int(max(r.steps for r in resp)),
                            "minres_iters": int(sum(r.minres_iters for r in resp)),
                            "max_rel_resid": float(max(r.max_rel_resid for r in resp))}
    out["unit"] = "s per converged eigenpair"
    return out


def plain_leg(mbl, torch):
    """The L=14 plain workload (h = 3, seed 0, the 10 pairs nearest the
    spectral midpoint, FP64): seconds per converged eigenpair on the GPU, the
    same unit as the oracle's dense solver in cpu_baseline."""
    from workloads import WORKLOADS, disorder_fields
    cfg = WORKLOADS["plain_L14"]
    f = disorder_fields(cfg["L"], cfg["h"], cfg["seeds"][0])
    b = mbl.Basis(cfg["L"])
    mbl.si_lanczos(b, f, 0.0, 2, seed=1)   # first-call setup (graph capture) outside the timing
    torch.cuda.synchronize()
    t = time.perf_counter()
    lo, hi, sg = mbl.sigma_midpoint(b, f, 1e-12)
    res = mbl.si_lanczos(b, f, sg, cfg["nev"], escale=max(abs(lo), abs(hi)), seed=7)
    mbl.twist_expect(b, res.evecs)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    progress(f"plain L=14 leg: {dt:.2f} s, {res.nconv} pairs")
    return {"L": cfg["L"], "nev": cfg["nev"], "h": cfg["h"], "value": round(dt / max(res.nconv, 1), 4),
            "unit": "s per converged eigenpair", "nconv": int(res.nconv), "seconds": round(dt, 3),
            "steps": int(res.steps), "minres_iters": int(res.minres_iters)}


def largest_leg(mbl, torch, steps=20):
    """The largest single-GPU workload (L=26, n = 10 400 600, h = 3.8, seed 0):
    device memory of a workspace against the linear model, apply throughput
    (one realization per launch, and 16 in lockstep), MINRES time per
    iteration in both precisions. Bounded: no converged eigenpair."""
    from workloads import WORKLOADS, disorder_fields
    cfg = WORKLOADS["largest_L26"]
    L = cfg["L"]
    h = disorder_fields(L, cfg["h"], cfg["seeds"][0])
    b = mbl.Basis(L)
    n = b.n
    out = {"L": L, "n": n, "h": cfg["h"], "lo_bits": b.lo_bits}
    free0 = torch.cuda.mem_get_info()[0]
    ws = mbl.Workspace(b, 70)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    out["workspace_mmax70_bytes"] = ws.bytes
    out["device_bytes_taken"] = int(free0 - free1)
    out["linear_model_bytes_8n(13+71)"] = 8 * n * (13 + 71)
    out["paper_model_bytes_8n(9+m)_m70"] = 8 * n * (9 + 70)
    t = time.perf_counter()
    lo, hi, sigma = mbl.sigma_midpoint(b, h, 1e-10)
    out["sigma"] = sigma
    out["sigma_seconds"] = round(time.perf_counter() - t, 3)
    progress(f"largest L=26: sigma {sigma:.6f} in {out['sigma_seconds']} s")
    g = torch.Generator(device="cuda").manual_seed(2)
    pairs = [(torch.randn(n, dtype=torch.float64, device="cuda", generator=g),
              torch.empty(n, dtype=torch.float64, device="cuda")) for _ in range(4)]
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for x, y in pairs:
        mbl.apply_H(b, h, sigma, x, y)
    e0.record(stream)
    for i in range(steps):
        x, y = pairs[i % 4]
        mbl.apply_H(b, h, sigma, x, y)
    e1.record(stream)
    torch.cuda.synchronize()
    us = e0.elapsed_time(e1) * 1e3 / steps
    out["apply_single"] = {"us": round(us, 2), "GBps": round(16.0 * n / us / 1e3, 1)}
    progress(f"largest L=26: single apply {us:.1f} us")
    del pairs
    R = 16
    bt = mbl.Batch(b, R)
    fields = [disorder_fields(L, cfg["h"], s) for s in range(R)]
    sig = [sigma] * R
    X = torch.randn((n, R), dtype=torch.float64, device="cuda", generator=g)
    Y = torch.empty_like(X)
    mbl.apply_H_batched(b, bt, fields, sig, X, Y)
    e0.record(stream)
    for _ in range(max(2, steps // 4)):
        mbl.apply_H_batched(b, bt, fields, sig, X, Y)
    e1.record(stream)
    torch.cuda.synchronize()
    us = e0.elapsed_time(e1) * 1e3 / max(2, steps // 4)
    out["apply_batched_R16"] = {"us": round(us, 2), "GBps": round(16.0 * n * R / us / 1e3, 1)}
    progress(f"largest L=26: batched R=16 apply {us:.1f} us")
    rhs = (X[:, 0] / X[:, 0].norm()).contiguous()
    for prec in ("fp64", "fp32_inner"):
        mbl.minres_solve(b, h, sigma, rhs, torch.zeros_like(rhs), tol=1e-300, kmax=200,
                         precision=prec, ws=ws)      # warm-up (graph capture)
        x = torch.zeros_like(rhs)
        torch.cuda.synchronize()
        t = time.perf_counter()
        _, info = mbl.minres_solve(b, h, sigma, rhs, x, tol=1e-300, kmax=200, precision=prec, ws=ws)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        out["minres_single_" + prec] = {"iters": int(info.iters),
                                        "us_per_iter": round(dt / max(info.iters, 1) * 1e6, 2)}
        progress(f"largest L=26: minres single {prec} {dt / max(info.iters, 1) * 1e6:.1f} us/iter")
    Bn = (X / X.norm(dim=0, keepdim=True)).contiguous()
    mbl.minres_solve_batched(b, bt, fields, sig, Bn, tol=1e-300, kmax=32)   # warm-up
    torch.cuda.synchronize()
    t = time.perf_counter()
    _, its, _, _ = mbl.minres_solve_batched(b, bt, fields, sig, Bn, tol=1e-300, kmax=32)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    it = int(its.max())
    out["minres_batched_R16_fp64"] = {"iters": it, "us_per_iter": round(dt / it * 1e6, 1),
                                      "us_per_realization_iter": round(dt / it / R * 1e6, 2)}
    progress(f"largest L=26: minres batched R=16 {dt / it * 1e6:.1f} us/iter")
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark measures one GPU (realizations are independent, "
                                   "so more GPUs would each run their own batches); use --gpus 1"}))
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
    # interleaved batch: element (i, r) at i * R + r. Successive steps rotate
    # over NPAIRS distinct (x, y) pairs, so the timed footprint is several
    # times the 256 MB last-level cache and no step finds its input there.
    g = torch.Generator(device="cuda").manual_seed(1)
    XS = [torch.randn((n, R), dtype=torch.float64, device=dev, generator=g) for _ in range(NPAIRS)]
    YS = [torch.empty_like(XS[0]) for _ in range(NPAIRS)]
    X, Y = XS[0], YS[0]
    batch = mbl.Batch(basis, R)
    tune.apply_schedule(batch, L, R, "fp64")
    stream = torch.cuda.current_stream()
    counter = [0]

    def step():
        i = counter[0] % NPAIRS
        counter[0] += 1
        mbl.apply_H_batched(basis, batch, fields, sigmas, XS[i], YS[i])

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

    progress(f"setup done: L={L} n={n} R={R} lo_bits={basis.lo_bits}")
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

    progress(f"batched apply: {achieved:.1f} GB/s ({avg_launch * 1e6:.1f} us per launch)")
    # attainable rate on this machine: a plain device copy of the same algorithmic
    # bytes (read 8nR, write 8nR), rotated over the same buffers
    ncopy = max(10, args.steps // 5)
    for i in range(NPAIRS):
        YS[i].copy_(XS[i])
    torch.cuda.synchronize()
    e0.record(stream)
    for k in range(ncopy):
        YS[k % NPAIRS].copy_(XS[k % NPAIRS])
    e1.record(stream)
    torch.cuda.synchronize()
    copy_gbs = bytes_per_launch / (e0.elapsed_time(e1) * 1e-3 / ncopy) / 1e9
    progress(f"device copy of the same bytes: {copy_gbs:.1f} GB/s")
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
        # a warm-up solve with the same arguments: the iteration blocks are
        # captured as a graph keyed on them, once per workspace
        mbl.minres_solve(basis, fields[0], sigmas[0], rhs, torch.zeros_like(rhs), tol=1e-300,
                         kmax=args.minres_iters, precision=prec, ws=ws)
        x = torch.zeros_like(rhs)
        torch.cuda.synchronize()
        t = time.perf_counter()
        _, info = mbl.minres_solve(basis, fields[0], sigmas[0], rhs, x, tol=1e-300,
                                   kmax=args.minres_iters, precision=prec, ws=ws)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        progress(f"minres single {prec}: {dt / max(info.iters, 1) * 1e6:.1f} us/iter")
        minres["single_" + prec] = {"iters": int(info.iters),
                                    "us_per_iter": round(dt / max(info.iters, 1) * 1e6, 2),
                                    "us_per_realization_iter": round(dt / max(info.iters, 1) * 1e6, 2),
                                    # ten n-vectors (z x 2, q x 3, d x 2, p, x, b): under the
                                    # 256 MB last-level cache at L=22
                                    "footprint_bytes": int(10 * n * (8 if prec == "fp64" else 4)),
                                    "cache_resident": True}
    Bn = (X / X.norm(dim=0, keepdim=True)).contiguous()
    for prec in ("fp64", "fp32_inner"):
        mbl.minres_solve_batched(basis, batch, fields, sigmas, Bn, tol=1e-300,
                                 kmax=max(1, args.minres_iters // 10), precision=prec)
        torch.cuda.synchronize()
        t = time.perf_counter()
        _, its, _, _ = mbl.minres_solve_batched(basis, batch, fields, sigmas, Bn, tol=1e-300,
                                               kmax=max(1, args.minres_iters // 10), precision=prec)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        it = int(its.max())
        progress(f"minres batched {prec}: {dt / max(it, 1) * 1e6:.1f} us/iter")
        minres["batched_" + prec] = {"iters": it, "realizations": R,
                                     "us_per_iter": round(dt / max(it, 1) * 1e6, 2),
                                     "us_per_realization_iter": round(dt / max(it, 1) / R * 1e6, 2),
                                     "footprint_bytes": int(18 * n * R * (8 if prec == "fp64" else 4)),
                                     "cache_resident": False}

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
                   "step": "one batched apply_H over all realizations (interleaved n x R)",
                   "xy_pairs_rotated": NPAIRS,
                   "timed_footprint_bytes": int(NPAIRS * 2 * 8 * n * R)},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic(headline_kernel(L, basis.lo_bits, R)),
                     "kernel": headline_kernel(L, basis.lo_bits, R),
                     "bytes_per_launch": bytes_per_launch, "avg_launch_us": round(avg_launch * 1e6, 3)},
        "attainable": {"copy_GBps": round(copy_gbs, 1),
                       "frac_of_copy": round(achieved / copy_gbs, 4)},
        "apply_single_realization": {"GBps": round(16.0 * n / single_s / 1e9, 1),
                                     "avg_launch_us": round(single_s * 1e6, 3),
                                     "footprint_bytes": int(16 * n), "cache_resident": True},
        "minres_L22": minres,
        "wall_s": round(wall, 3),
    }
    tr = out["roofline"]["traffic"]
    if tr:
        out["roofline"]["traffic_GBps"] = round(tr / avg_launch / 1e9, 1)
        out["roofline"]["amplification"] = round(tr / bytes_per_launch, 3)
    if not args.no_eig:
        out["sec_per_eigenpair"] = eig_leg(mbl, torch, args.eig_L, args.eig_nev, args.eig_R,
                                           args.eig_batched_mixed)
        out["sec_per_eigenpair_plain_L14"] = plain_leg(mbl, torch)
    if args.largest:
        out["largest_L26"] = largest_leg(mbl, torch)
    if not args.no_cpu:
        progress("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(fields, sigmas, L)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
