"""Small studies built on the library (beyond the hot path itself).

* ``precond``: MINRES iterations and time to solve (H - sigma) x = b at the
  spectral midpoint with the identity, Jacobi and row-norm preconditioners
  (the comparison of Sec. II / Sec. IV A: iterations against L for h = 3, 4).
* ``memory``: device bytes of a workspace against L, next to the linear model
  8 n (12 + mmax + 1) and the paper's 8 n (9 + m) (Sec. IV A).

    python -m paper_2203_09732_amd.studies precond --L 12 14 16 18 20 --h 3 4 --seeds 0 1
    python -m paper_2203_09732_amd.studies memory --L 12 14 16 18 20 22 24 26

One JSON object per line on stdout.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time


def precond_iterations(Ls, hs, seeds, kinds=("id", "jacobi", "row"), tol=1e-12, kmax_per_n=30):
    import torch

    import paper_2203_09732_amd as mbl
    from workloads import disorder_fields, start_vector
    for L in Ls:
        b = mbl.Basis(L)
        ws = mbl.Workspace(b, 0)
        for h in hs:
            for seed in seeds:
                f = disorder_fields(L, h, seed)
                _, _, sigma = mbl.sigma_midpoint(b, f, 1e-12)
                rhs = torch.as_tensor(start_vector(b.n, seed), device="cuda")
                rhs /= torch.linalg.norm(rhs)
                for kind in kinds:
                    x = torch.zeros_like(rhs)
                    torch.cuda.synchronize()
                    t = time.perf_counter()
                    _, info = mbl.minres_solve(b, f, sigma, rhs, x, tol=tol, kmax=kmax_per_n * b.n,
                                               precond=kind, ws=ws)
                    torch.cuda.synchronize()
                    yield {"study": "precond", "L": L, "n": b.n, "h": h, "seed": seed,
                           "precond": kind, "iters": info.iters, "iters_per_n": info.iters / b.n,
                           "seconds": round(time.perf_counter() - t, 3),
                           "converged": info.status == 0, "true_res": info.true_res}


def memory_curve(Ls, mmax=130):
    import paper_2203_09732_amd as mbl
    for L in Ls:
        b = mbl.Basis(L)
        ws = mbl.Workspace(b, mmax)
        yield {"study": "memory", "L": L, "n": b.n, "mmax": mmax, "workspace_bytes": ws.bytes,
               "model_8n(12+mmax+1)": 8 * b.n * (12 + mmax + 1),
               "paper_model_8n(9+m)": 8 * b.n * (9 + mmax)}
        del ws


def main(argv=None):
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    ap = argparse.ArgumentParser()
    ap.add_argument("study", choices=["precond", "memory"])
    ap.add_argument("--L", type=int, nargs="+", default=[12, 14, 16, 18])
    ap.add_argument("--h", type=float, nargs="+", default=[3.0, 4.0])
    ap.add_argument("--seeds", type=int, nargs="+", default=[0, 1])
    ap.add_argument("--mmax", type=int, default=130)
    a = ap.parse_args(argv)
    rows = (precond_iterations(a.L, a.h, a.seeds) if a.study == "precond"
            else memory_curve(a.L, a.mmax))
    for r in rows:
        print(json.dumps(r), flush=True)


if __name__ == "__main__":
    main()
