"""Autotuner for the row kernels' block split.

The sector basis is stored as (high bits, low bits) blocks; the number of low
bits sets the block size, which trades lane use in a wavefront against the
cache footprint of the neighbour gathers (bonds inside the low bits hit rows
of the same block, bonds in the high bits reach other blocks). The best split
depends on L, on the batch width R and on the vector precision, so it is
measured: each candidate split with a compiled instance is timed on the GPU
and the fastest is cached in tuning.json, keyed by GPU architecture.

    python -m paper_2203_09732_amd.tune --L 22 --R 32 [--precision fp32]
"""
from __future__ import annotations

import argparse
import json
import os
import time

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(HERE, "tuning.json")

# splits with compiled instances (the library's default split first)
CANDIDATES = {
    12: [9], 14: [10, 7], 16: [10, 8], 18: [12, 9], 20: [13, 11, 9],
    22: [13, 11, 9], 24: [13, 11, 9], 26: [13, 11, 9], 28: [13], 30: [13], 32: [13],
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


def best_lo_bits(L: int, R: int, precision: str = "fp64") -> int:
    """Cached best split for (arch, L, R, precision); 0 (library default) if unknown."""
    try:
        entry = load_cache().get(_arch(), {}).get(_key(L, R, precision))
    except Exception:
        entry = None
    return int(entry["lo_bits"]) if entry else 0


def time_batched_apply(L: int, R: int, lo_bits: int, precision: str = "fp64", reps: int = 30,
                       seed: int = 0) -> float:
    """Seconds per batched apply (R realizations) with the given split."""
    import numpy as np
    import torch

    import paper_2203_09732_amd as mbl
    from workloads import disorder_fields

    b = mbl.Basis(L, lo_bits)
    dt = torch.float64 if precision == "fp64" else torch.float32
    bt = mbl.Batch(b, R)
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


def tune(L: int, R: int, precision: str = "fp64", reps: int = 30, write: bool = True) -> dict:
    from math import comb
    n = comb(L, L // 2)
    esize = 8 if precision == "fp64" else 4
    results = {}
    for lo in CANDIDATES.get(L, [0]):
        try:
            t = time_batched_apply(L, R, lo, precision, reps)
        except Exception as e:       # split not valid for this R (LDS) etc.
            results[lo] = {"error": str(e)}
            continue
        results[lo] = {"seconds": t, "GBps": 2 * esize * n * R / t / 1e9}
    ok = {k: v for k, v in results.items() if "seconds" in v}
    if not ok:
        return {"results": results}
    best = min(ok, key=lambda k: ok[k]["seconds"])
    entry = {"lo_bits": best, "GBps": round(ok[best]["GBps"], 1), "when": time.strftime("%Y-%m-%d"),
             "candidates": {str(k): round(v.get("GBps", 0.0), 1) for k, v in results.items()}}
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
                out = tune(L, R, p, a.reps)
                print(json.dumps({"L": L, "R": R, "precision": p, **out.get("best", {}),
                                  "all": {str(k): v for k, v in out["results"].items()}}), flush=True)
