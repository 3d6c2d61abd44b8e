"""Autotuner for the batched kernels' block split and launch schedule.

The sector basis is stored as (high bits, low bits) blocks; the number of low
bits sets the block size, which trades lane use in a wavefront against the
cache footprint of the neighbour gathers (bonds inside the low bits hit rows
of the same block, bonds in the high bits reach other blocks). The launch
schedule of a batch workspace adds three knobs: the number of workgroups of
the row kernels, the MINRES iterations per captured graph, and the MINRES
iterations per d/x pass. The best values depend on L, on the batch width R
and on the vector precision, so they are measured, in two stages: every
(split, grid) pair is timed on the batched apply; then, at the fastest pair,
every (graph length, d/x pass length) pair is timed on batched MINRES
iterations. The winner is cached in tuning.json, keyed by GPU architecture.

    python -m paper_2203_09732_amd.tune --L 22 --R 32 [--precision fp32]
"""
from __future__ import annotations

import argparse
import json
import os
import time

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(HERE, "tuning.json")

# splits with compiled instances (the library's default split first); at
# R = 32 the split 10 of L = 14, 16 and 22 takes the block-staged product
CANDIDATES = {
    12: [9], 14: [10, 7], 16: [10, 8], 18: [12, 9], 20: [13, 11, 9],
    22: [13, 11, 10, 9], 24: [13, 11, 9], 26: [13, 11, 9], 28: [13], 30: [13], 32: [13],
}


def _arch() -> str:
    import torch
    p = torch.cuda.get_device_properties(0)
    return getattr(p, "gcnArchName", p.name).split(":")[0]


def _key(L: int, R: int, precision: str) -> str:
    return f"L{L}_R{R}_{precision}"


def load_cache() -> dict:
    if os.path.exists(CACHE):
        with open(CACHE) as fh:
            return json.load(fh)
    return {}


GRIDS = (0, 128, 256, 384, 512)     # row-kernel workgroups; 0: one per compute unit
GRAPH_ITERS = (8, 16, 32)            # MINRES iterations per captured graph
DX_GROUPS = (1, 2, 4)                # MINRES iterations per d/x pass


def _entry(L: int, R: int, precision: str):
    try:
        return load_cache().get(_arch(), {}).get(_key(L, R, precision))
    except Exception:
        return None


def best_lo_bits(L: int, R: int, precision: str = "fp64") -> int:
    """Cached best split for (arch, L, R, precision); 0 (library default) if unknown."""
    entry = _entry(L, R, precision)
    return int(entry["lo_bits"]) if entry else 0


def best_schedule(L: int, R: int, precision: str = "fp64") -> tuple[int, int, int]:
    """Cached (grid, graph_iters, dx_group); zeros (library defaults) if unknown."""
    entry = _entry(L, R, precision)
    if not entry:
        return (0, 0, 0)
    return (int(entry.get("grid", 0)), int(entry.get("graph_iters", 0)),
            int(entry.get("dx_group", 0)))


def apply_schedule(batch, L: int, R: int, precision: str = "fp64") -> None:
    """Give a batch workspace the cached schedule for (L, R, precision)."""
    batch.set_schedule(*best_schedule(L, R, precision))


def time_batched_apply(L: int, R: int, lo_bits: int, precision: str = "fp64", reps: int = 30,
                       seed: int = 0, grid: int = 0) -> float:
    """Seconds per batched apply (R realizations) with the given split and grid."""
    import numpy as np
    import torch

    import paper_2203_09732_amd as mbl
    from workloads import disorder_fields

    b = mbl.Basis(L, lo_bits)
    dt = torch.float64 if precision == "fp64" else torch.float32
    bt = mbl.Batch(b, R)
    bt.set_schedule(grid, 0, 0)
    fields = [disorder_fields(L, 3.5, seed + r) for r in range(R)]
    sig = np.zeros(R)
    g = torch.Generator(device="cuda").manual_seed(seed)
    X = torch.randn((b.n, R), dtype=dt, device="cuda", generator=g)
    Y = torch.empty_like(X)
    for _ in range(3):
        mbl.apply_H_batched(b, bt, fields, sig, X, Y)
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        mbl.apply_H_batched(b, bt, fields, sig, X, Y)
    e1.record(s)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) * 1e-3 / reps


def time_batched_minres(L: int, R: int, lo_bits: int, grid: int, graph_iters: int, dx_group: int,
                        iters: int = 193, seed: int = 0) -> float:
    """Seconds per FP64 batched MINRES iteration (R realizations) with the
    given split and schedule: a solve of exactly `iters` iterations
    (tolerance 1e-300; 193 = 1 + 3 x 64, so that after the first iteration
    every chunk is whole graphs for each graph length), after one untimed solve
    that captures the graphs."""
    import numpy as np
    import torch

    import paper_2203_09732_amd as mbl
    from workloads import disorder_fields

    b = mbl.Basis(L, lo_bits)
    bt = mbl.Batch(b, R)
    bt.set_schedule(grid, graph_iters, dx_group)
    fields = [disorder_fields(L, 3.5, seed + r) for r in range(R)]
    sig = np.zeros(R)
    g = torch.Generator(device="cuda").manual_seed(seed)
    rhs = torch.randn((b.n, R), dtype=torch.float64, device="cuda", generator=g)
    x = torch.zeros_like(rhs)
    mbl.minres_solve_batched(b, bt, fields, sig, rhs, x, tol=1e-300, kmax=iters)
    torch.cuda.synchronize()
    t = time.perf_counter()
    _, its, _, _ = mbl.minres_solve_batched(b, bt, fields, sig, rhs, x, tol=1e-300, kmax=iters)
    torch.cuda.synchronize()
    return (time.perf_counter() - t) / max(int(its.max()), 1)


def tune(L: int, R: int, precision: str = "fp64", reps: int = 30, write: bool = True,
         log=None) -> dict:
    from math import comb
    n = comb(L, L // 2)
    esize = 8 if precision == "fp64" else 4
    results = {}
    for lo in CANDIDATES.get(L, [0]):
        for grid in GRIDS:
            key = f"lo{lo}_g{grid}"
            try:
                t = time_batched_apply(L, R, lo, precision, reps, grid=grid)
            except Exception as e:       # split not valid for this R (LDS) etc.
                results[key] = {"error": str(e)}
                continue
            results[key] = {"lo_bits": lo, "grid": grid, "seconds": t,
                            "GBps": 2 * esize * n * R / t / 1e9}
            if log:
                log(f"apply L={L} R={R} {precision} lo_bits={lo} grid={grid}: "
                    f"{results[key]['GBps']:.1f} GB/s")
    ok = {k: v for k, v in results.items() if "seconds" in v}
    if not ok:
        return {"results": results}
    best = min(ok, key=lambda k: ok[k]["seconds"])
    lo_b, grid_b = ok[best]["lo_bits"], ok[best]["grid"]
    minres = {}
    # the MINRES knobs are timed on FP64 iterations (FP32-inner solves stop on
    # their own inner tolerance, not after a fixed count); FP32 keeps 16 / 4
    for gi in (GRAPH_ITERS if precision == "fp64" else (16,)):
        for dx in (DX_GROUPS if precision == "fp64" else (4,)):
            t = time_batched_minres(L, R, lo_b, grid_b, gi, dx) if precision == "fp64" else 0.0
            minres[f"graph{gi}_dx{dx}"] = {"graph_iters": gi, "dx_group": dx, "us_per_iter": t * 1e6}
            if log:
                log(f"minres L={L} R={R} {precision} graph_iters={gi} dx_group={dx}: "
                    f"{t * 1e6:.1f} us per iteration")
    mbest = min(minres, key=lambda k: minres[k]["us_per_iter"])
    entry = {"lo_bits": lo_b, "grid": grid_b, "graph_iters": minres[mbest]["graph_iters"],
             "dx_group": minres[mbest]["dx_group"], "GBps": round(ok[best]["GBps"], 1),
             "minres_us_per_iter": round(minres[mbest]["us_per_iter"], 2),
             "when": time.strftime("%Y-%m-%d"),
             "candidates": {k: round(v.get("GBps", 0.0), 1) for k, v in results.items()},
             "minres_candidates": {k: round(v["us_per_iter"], 2) for k, v in minres.items()}}
    if write:
        cache = load_cache()
        cache.setdefault(_arch(), {})[_key(L, R, precision)] = entry
        with open(CACHE, "w") as fh:
            json.dump(cache, fh, indent=1, sort_keys=True)
    return {"results": results, "best": entry}


if __name__ == "__main__":
    import sys
    sys.path.insert(0, os.path.dirname(HERE))
    ap = argparse.ArgumentParser()
    ap.add_argument("--L", type=int, nargs="+", default=[22])
    ap.add_argument("--R", type=int, nargs="+", default=[32])
    ap.add_argument("--precision", nargs="+", default=["fp64"])
    ap.add_argument("--reps", type=int, default=30)
    a = ap.parse_args()
    for L in a.L:
        for R in a.R:
            for p in a.precision:
                out = tune(L, R, p, a.reps, log=lambda m: print(m, file=sys.stderr, flush=True))
                print(json.dumps({"L": L, "R": R, "precision": p, **out.get("best", {})}),
                      flush=True)
