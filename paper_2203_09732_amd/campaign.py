"""Disorder campaigns: many realizations of uneven chain length.

Two ways to run them:

* ``persistent`` (default): the realizations go to the library's problem-array
  call (mbl_si_lanczos_problems) in chunks of up to ``chunk`` realizations of
  any mix of L; realizations with L <= 16 are solved in one persistent launch
  per chunk, a workgroup per realization, sigma = (E_min + E_max)/2
  (Sec. IV A) included, and the longer ones in streaming batches of up to 32
  lanes inside the same call (each lane runs its own realization's Lanczos
  steps and takes the next realization when its own has converged);
* ``lockstep``: realizations are grouped by L and each group is solved in
  batches of R realizations (a power of two, as large as the kernels' LDS
  budget allows for that L) by the lockstep shift-invert Lanczos, after sigma
  has been found for each realization. A batch that is not full is padded
  with copies of its last realization, whose results are dropped. Within a
  chain length the realizations are ordered by their mean square field (the
  cost proxy the library's problem-array call uses too).

One JSON line per realization is appended to an optional results file;
realizations already present there are skipped, so an interrupted campaign
resumes where it stopped (at chunk or batch granularity).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from dataclasses import dataclass

import numpy as np

from . import Basis, Batch, si_lanczos_batched, si_lanczos_problems, sigma_midpoint
from . import tune, twist_expect_batched

MAX_R = 32


@dataclass
class Task:
    index: int
    L: int
    h: float
    fields: np.ndarray


def widest_batch(L: int, want: int) -> int:
    """Largest power of two <= min(want, 32) whose field tables fit the LDS budget."""
    R = 2
    while R * 2 <= min(max(want, 2), MAX_R) and (R * 2) * 16 * ((L + 3) // 4) * 8 <= 30 * 1024:
        R *= 2
    return R


def _done_indices(path):
    if not path or not os.path.exists(path):
        return set()
    out = set()
    with open(path) as fh:
        for line in fh:
            try:
                out.add(int(json.loads(line)["index"]))
            except Exception:
                continue
    return out


def run(tasks, nev: int, results_path: str | None = None, precision: str = "fp64",
        minres_tol: float = 1e-12, eig_tol: float = 1e-10, gap_tol: float = 1e-5,
        max_R: int = MAX_R, log=print, mode: str = "persistent", chunk: int = 1024):
    """Solve every task; returns the list of per-realization records."""
    done = _done_indices(results_path)
    todo = [t for t in tasks if t.index not in done]
    if mode == "persistent":
        if precision != "fp64":
            raise ValueError("the persistent form runs FP64")
        return _run_persistent(todo, nev, results_path, minres_tol, eig_tol, gap_tol, chunk, log)
    return _run_lockstep(todo, nev, results_path, precision, minres_tol, eig_tol, gap_tol, max_R,
                         log)


def _run_persistent(todo, nev, results_path, minres_tol, eig_tol, gap_tol, chunk, log):
    records = []
    for start in range(0, len(todo), chunk):
        part = todo[start:start + chunk]
        t0 = time.perf_counter()
        st, res = si_lanczos_problems([dict(L=t.L, h=t.fields, nev=nev) for t in part],
                                      minres_tol=minres_tol, eig_tol=eig_tol, gap_tol=gap_tol,
                                      seed=1234 + start)
        t_total = time.perf_counter() - t0
        for t, r in zip(part, res):
            rec = {
                "index": t.index, "L": t.L, "h": t.h, "sigma": r.sigma,
                "evals": r.evals.tolist(), "resid": r.resid.tolist(),
                "z_re": np.real(r.z).tolist(), "z_im": np.imag(r.z).tolist(),
                "steps": r.steps, "nconv": r.nconv, "status": r.status,
                "minres_iters": r.minres_iters, "mode": "persistent",
                "call_realizations": len(part), "call_seconds": t_total, "precision": "fp64",
            }
            records.append(rec)
            if results_path:
                with open(results_path, "a") as fh:
                    fh.write(json.dumps(rec) + "\n")
        if log:
            Ls = sorted({t.L for t in part})
            log(f"persistent call: {len(part)} realizations (L in {Ls}) {t_total:.1f}s, "
                f"pairs converged {sum(r.nconv for r in res)} of {nev * len(part)}")
    return records


def _run_lockstep(todo, nev, results_path, precision, minres_tol, eig_tol, gap_tol, max_R, log):
    import torch
    records = []
    for L in sorted({t.L for t in todo}):
        # similar disorder strength in one batch: a batch runs as many MINRES
        # iterations per step as its slowest realization needs
        group = sorted((t for t in todo if t.L == L), key=lambda t: float(np.mean(t.fields ** 2)))
        R = widest_batch(L, min(max_R, len(group)))
        while True:       # narrower batches if the split's tables leave too little LDS
            basis = Basis(L, tune.best_lo_bits(L, R, precision))
            mmax = min(basis.n, 3 * nev + 40)
            try:
                batch = Batch(basis, R, mmax=mmax, nevmax=nev)
                tune.apply_schedule(batch, L, R, precision)
                break
            except Exception:
                if R == 2:
                    raise
                R //= 2
        for start in range(0, len(group), R):
            chunk = group[start:start + R]
            real = len(chunk)
            padded = chunk + [chunk[-1]] * (R - real)
            t0 = time.perf_counter()
            sig, esc = [], []
            for t in padded:
                lo, hi, sg = sigma_midpoint(basis, t.fields, 1e-12)
                sig.append(sg)
                esc.append(max(abs(lo), abs(hi)))
            t_sigma = time.perf_counter() - t0
            res = si_lanczos_batched(basis, batch, [t.fields for t in padded], sig, nev, mmax=mmax,
                                     minres_tol=minres_tol, eig_tol=eig_tol, gap_tol=gap_tol,
                                     escale=esc, seed=1234 + start, precision=precision)
            z = twist_expect_batched(basis, batch, res.evecs)
            torch.cuda.synchronize()
            t_total = time.perf_counter() - t0
            for r, t in enumerate(chunk):
                rec = {
                    "index": t.index, "L": L, "h": t.h, "sigma": sig[r], "E_min_max_scale": esc[r],
                    "evals": res.evals[r].tolist(), "resid": res.resid[r].tolist(),
                    "z_re": np.real(z[r]).tolist(), "z_im": np.imag(z[r]).tolist(),
                    "steps": int(res.steps[r]), "nconv": int(res.nconv[r]),
                    "batch_R": R, "batch_seconds": t_total, "sigma_seconds": t_sigma,
                    "batch_minres_iters": res.minres_iters, "precision": precision,
                    "mode": "lockstep",
                }
                records.append(rec)
                if results_path:
                    with open(results_path, "a") as fh:
                        fh.write(json.dumps(rec) + "\n")
            if log:
                log(f"L={L} batch {start // R} R={R} ({real} real) {t_total:.1f}s "
                    f"steps={list(res.steps[:real])} nconv={list(res.nconv[:real])}")
    return records


def main(argv=None):
    """Run the mixed-size campaign of seeded realizations 0 .. count-1 (chain
    length and disorder strength drawn per realization) and print one summary
    line per chain length.

        python -m paper_2203_09732_amd.campaign --count 512 --nev 6 --out results.jsonl
    """
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    from workloads import batched_realizations
    ap = argparse.ArgumentParser()
    ap.add_argument("--count", type=int, default=512)
    ap.add_argument("--nev", type=int, default=6)
    ap.add_argument("--out", default=None, help="JSON lines, one per realization (resumable)")
    ap.add_argument("--max-R", type=int, default=MAX_R)
    ap.add_argument("--precision", default="fp64")
    ap.add_argument("--mode", default="persistent", choices=["persistent", "lockstep"])
    ap.add_argument("--chunk", type=int, default=1024,
                    help="realizations per problem-array call (persistent mode)")
    a = ap.parse_args(argv)
    tasks = [Task(r.index, r.L, r.h, r.fields) for r in batched_realizations(a.count)]
    t0 = time.perf_counter()
    recs = run(tasks, a.nev, results_path=a.out, precision=a.precision, max_R=a.max_R,
               log=lambda m: print(m, flush=True), mode=a.mode, chunk=a.chunk)
    wall = time.perf_counter() - t0
    by_L = {}
    for rec in recs:
        d = by_L.setdefault(rec["L"], {"realizations": 0, "pairs": 0, "batches": set(), "seconds": 0.0,
                                       "minres_iters": 0})
        d["realizations"] += 1
        d["pairs"] += rec["nconv"]
        if rec["mode"] == "lockstep" and (rec["batch_R"], rec["batch_seconds"]) not in d["batches"]:
            d["batches"].add((rec["batch_R"], rec["batch_seconds"]))
            d["seconds"] += rec["batch_seconds"]
        d["minres_iters"] += rec.get("minres_iters", 0)
    for L, d in sorted(by_L.items()):
        row = {"L": L, "realizations": d["realizations"], "converged_pairs": d["pairs"]}
        if a.mode == "lockstep":
            row.update(seconds=round(d["seconds"], 2), s_per_pair=round(d["seconds"] / max(d["pairs"], 1), 4))
        else:
            row.update(minres_iters=d["minres_iters"])
        print(json.dumps(row), flush=True)
    pairs = sum(d["pairs"] for d in by_L.values())
    print(json.dumps({"mode": a.mode, "total_seconds": round(wall, 2), "realizations": len(recs),
                      "converged_pairs": pairs, "s_per_pair": round(wall / max(pairs, 1), 4)}),
          flush=True)


if __name__ == "__main__":
    main()
