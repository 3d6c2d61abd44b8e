"""Small studies built on the library (beyond the hot path itself).

* ``precond``: MINRES iterations and time to solve (H - sigma) x = b at the
  spectral midpoint with the identity, Jacobi and row-norm preconditioners
  (the comparison of Sec. II / Sec. IV A: iterations against L for h = 3, 4).
* ``memory``: device bytes of a workspace against L, next to the linear model
  8 n (13 + mmax + 1) and the paper's 8 n (9 + m) (Sec. IV A).
* ``eig``: one full shift-invert Lanczos run (sigma at the spectral midpoint,
  the nev pairs nearest it, MINRES tol 1e-12, eig_tol 1e-10), its time per
  converged eigenpair, steps and MINRES iterations (set MBL_VERBOSE=1 for a
  line per Lanczos step).

    python -m paper_2203_09732_amd.studies precond --L 12 14 16 18 20 --h 3 4 --seeds 0 1
    python -m paper_2203_09732_amd.studies memory --L 12 14 16 18 20 22 24 26
    MBL_VERBOSE=1 python -m paper_2203_09732_amd.studies eig --L 22 --h 3.5 --nev 4

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
               "model_8n(13+mmax+1)": 8 * b.n * (13 + mmax + 1),
               "paper_model_8n(9+m)": 8 * b.n * (9 + mmax)}
        del ws


def eigen_run(L, h, seed, nev, precision="fp64"):
    import torch

    import paper_2203_09732_amd as mbl
    from workloads import disorder_fields
    b = mbl.Basis(L)
    f = disorder_fields(L, h, seed)
    t0 = time.perf_counter()
    lo, hi, sigma = mbl.sigma_midpoint(b, f, 1e-12)
    t_sigma = time.perf_counter() - t0
    escale = max(abs(lo), abs(hi))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = mbl.si_lanczos(b, f, sigma, nev, escale=escale, seed=seed, precision=precision)
    z = mbl.twist_expect(b, res.evecs)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    yield {"study": "eig", "L": L, "n": b.n, "h": h, "seed": seed, "nev": nev,
           "precision": precision, "sigma": sigma, "sigma_seconds": round(t_sigma, 3),
           "seconds": round(dt, 2), "nconv": int(res.nconv), "steps": int(res.steps),
           "minres_iters": int(res.minres_iters),
           "minres_iters_per_step_per_n": res.minres_iters / max(res.steps, 1) / b.n,
           "s_per_pair": round(dt / max(res.nconv, 1), 2),
           "max_resid_over_escale": float(max(res.resid) / escale),
           "evals": [float(e) for e in res.evals], "abs_z": [float(abs(v)) for v in z]}


def main(argv=None):
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    ap = argparse.ArgumentParser()
    ap.add_argument("study", choices=["precond", "memory", "eig"])
    ap.add_argument("--L", type=int, nargs="+", default=[12, 14, 16, 18])
    ap.add_argument("--h", type=float, nargs="+", default=[3.0, 4.0])
    ap.add_argument("--seeds", type=int, nargs="+", default=[0, 1])
    ap.add_argument("--mmax", type=int, default=130)
    ap.add_argument("--nev", type=int, default=4)
    ap.add_argument("--precision", default="fp64")
    a = ap.parse_args(argv)
    if a.study == "precond":
        rows = precond_iterations(a.L, a.h, a.seeds)
    elif a.study == "memory":
        rows = memory_curve(a.L, a.mmax)
    else:
        rows = (r for L in a.L for r in eigen_run(L, a.h[0], a.seeds[0], a.nev, a.precision))
    for r in rows:
        print(json.dumps(r), flush=True)


if __name__ == "__main__":
    main()
