"""Small studies built on the library (beyond the hot path itself).

* ``precond``: MINRES iterations and time to solve (H - sigma) x = b at the
  spectral midpoint with the identity, Jacobi and row-norm preconditioners
  (the comparison of Sec. II / Sec. IV A: iterations against L for h = 3, 4).
* ``memory``: device memory a workspace takes against L, measured as the
  drop of the device's free memory (hipMemGetInfo) across its creation, next
  to the library's own count, the linear model 8 n (13 + mmax + 1) and the
  paper's 8 n (9 + m) (Sec. IV A).
* ``scan``: the disorder scan of Sec. IV: for each (L, h), R realizations
  solved together in the batched form (the nev pairs nearest each one's
  spectral midpoint), then per realization the mean level-spacing ratio,
  the mean half-chain entanglement entropy and the mean |z|^2 over its
  eigenstates; the row reports their mean and standard deviation over
  realizations, next to the GOE and Poisson ratios and the random-state entropy of Sec. IV B, and
  the per-realization values (with sigma and the eigenvalues).
* ``grad``: eigenpair derivatives for many realizations (the L = 20, h = 3,
  16 realizations, 4 pairs form): the nev pairs nearest each realization's
  spectral midpoint from one problem-array call, then dE/dh_j and
  d|z|^2/dh_j for every site and every converged pair (Hellmann-Feynman and
  one adjoint MINRES solve, Sec. III), with the two sum rules that hold
  exactly in the S^z = 0 sector (a uniform field shift changes neither the
  eigenvectors nor, summed over sites, the energy): sum_j dE/dh_j = 0 and
  sum_j d|z|^2/dh_j = 0; seconds per pair for both parts.
* ``mixed``: the mixed-precision form against FP64 on the same realization
  (config 3's deliverable at a size one run can hold): SI-Lanczos with FP64
  MINRES and with FP32-inner MINRES from the same start vector; the
  eigenvalue differences |E_32 - E_64| / max(|E_64|, 1), the eigenvector
  overlap deficits 1 - |<u_32, u_64>|, the twist differences, the explicit
  residuals of both, and seconds per pair of both.
* ``eig``: one full shift-invert Lanczos run (sigma at the spectral midpoint,
  the nev pairs nearest it, MINRES tol 1e-12, eig_tol 1e-10), its time per
  converged eigenpair, steps and MINRES iterations (set MBL_VERBOSE=1 for a
  line per Lanczos step).

    python -m paper_2203_09732_amd.studies precond --L 12 14 16 18 20 --h 3 4 --seeds 0 1
    python -m paper_2203_09732_amd.studies memory --L 12 14 16 18 20 22 24 26
    MBL_VERBOSE=1 python -m paper_2203_09732_amd.studies eig --L 22 --h 3.5 --nev 4
    python -m paper_2203_09732_amd.studies grad --L 20 --h 3 --R 16 --nev 4
    python -m paper_2203_09732_amd.studies mixed --L 20 --h 3.5 --nev 4

One JSON object per line on stdout.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np


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
    import torch

    import paper_2203_09732_amd as mbl
    mbl.Workspace(mbl.Basis(8), 2)        # first allocations of the process outside the count
    for L in Ls:
        b = mbl.Basis(L)
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        ws = mbl.Workspace(b, mmax)
        torch.cuda.synchronize()
        free1 = torch.cuda.mem_get_info()[0]
        yield {"study": "memory", "L": L, "n": b.n, "mmax": mmax,
               "device_bytes_taken": int(free0 - free1), "workspace_bytes": ws.bytes,
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


def mixed_study(L, h, seed, nev):
    import torch

    import paper_2203_09732_amd as mbl
    from workloads import disorder_fields
    b = mbl.Basis(L)
    f = disorder_fields(L, h, seed)
    lo, hi, sigma = mbl.sigma_midpoint(b, f, 1e-12)
    escale = max(abs(lo), abs(hi))
    out = {"study": "mixed", "L": L, "n": b.n, "h": h, "seed": seed, "nev": nev, "sigma": sigma,
           "escale": escale}
    res = {}
    for prec in ("fp64", "fp32_inner"):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = mbl.si_lanczos(b, f, sigma, nev, escale=escale, seed=seed, precision=prec)
        z = mbl.twist_expect(b, r.evecs)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        res[prec] = (r, z)
        out[prec] = {"seconds": round(dt, 2), "s_per_pair": round(dt / max(r.nconv, 1), 3),
                     "nconv": int(r.nconv), "steps": int(r.steps),
                     "minres_iters": int(r.minres_iters),
                     "max_rel_resid": float(max(r.resid) / escale)}
    (r64, z64), (r32, z32) = res["fp64"], res["fp32_inner"]
    if r64.nconv == nev and r32.nconv == nev:
        ov = torch.abs(torch.sum(r64.evecs * r32.evecs, dim=0)).cpu().numpy()
        out["max_rel_dE"] = float(np.max(np.abs(r32.evals - r64.evals) /
                                         np.maximum(np.abs(r64.evals), 1.0)))
        out["max_overlap_deficit"] = float(np.max(1.0 - ov))
        out["max_dz"] = float(np.max(np.abs(z32 - z64)))
    out["time_ratio_fp32_over_fp64"] = round(out["fp32_inner"]["seconds"] / out["fp64"]["seconds"], 3)
    yield out


def grad_study(L, h, R=16, nev=4, first_seed=0, tol=1e-12):
    import torch

    import paper_2203_09732_amd as mbl
    from workloads import disorder_fields
    fields = [disorder_fields(L, h, first_seed + r) for r in range(R)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st, res = mbl.si_lanczos_problems([dict(L=L, h=f, nev=nev) for f in fields], seed=first_seed)
    torch.cuda.synchronize()
    t_eig = time.perf_counter() - t0
    b = mbl.Basis(L)
    ws = mbl.Workspace(b, 0)
    rows, npairs, t_adj = [], 0, 0.0
    for r, (f, p) in enumerate(zip(fields, res)):
        pairs = []
        for t in range(len(p.evals) if p.status == 0 else 0):   # converged realizations
            psi = p.evecs[:, t].contiguous()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            dE, dz2, z, info = mbl.eig_grad(b, f, float(p.evals[t]), psi, tol=tol, ws=ws)
            torch.cuda.synchronize()
            t_adj += time.perf_counter() - t1
            npairs += 1
            pairs.append({"E": float(p.evals[t]), "abs_z": abs(z), "adjoint_iters": int(info.iters),
                          "adjoint_status": int(info.status),
                          "sum_dE": float(dE.sum()), "sum_dz2": float(dz2.sum()),
                          "max_abs_dz2": float(np.abs(dz2).max()),
                          "dE": [float(v) for v in dE], "dz2": [float(v) for v in dz2]})
        rows.append({"study": "grad", "L": L, "h": h, "seed": first_seed + r, "sigma": p.sigma,
                     "status": p.status, "nconv": p.nconv, "steps": p.steps, "pairs": pairs})
        yield rows[-1]
    yield {"study": "grad_summary", "L": L, "n": b.n, "h": h, "R": R, "nev": nev,
           "converged_pairs": npairs, "eig_seconds": round(t_eig, 2),
           "eig_s_per_pair": round(t_eig / max(npairs, 1), 3),
           "adjoint_seconds": round(t_adj, 2), "adjoint_s_per_pair": round(t_adj / max(npairs, 1), 3),
           "max_abs_sum_dE": max((abs(q["sum_dE"]) for r_ in rows for q in r_["pairs"]),
                                 default=float("nan")),
           "max_rel_sum_dz2": max((abs(q["sum_dz2"]) / max(1.0, q["max_abs_dz2"])
                                   for r_ in rows for q in r_["pairs"]), default=float("nan"))}


def disorder_scan(Ls, hs, R=32, nev=20, first_seed=0):
    import math

    import numpy as np
    import torch

    import paper_2203_09732_amd as mbl
    from paper_2203_09732_amd import tune
    from workloads import disorder_fields
    for L in Ls:
        b = mbl.Basis(L, tune.best_lo_bits(L, R, "fp64"))
        mmax = min(b.n, 3 * nev + 40)
        bt = mbl.Batch(b, R, mmax=mmax, nevmax=nev)
        tune.apply_schedule(bt, L, R, "fp64")
        for h in hs:
            fields = [disorder_fields(L, h, first_seed + r) for r in range(R)]
            t0 = time.perf_counter()
            sig, esc = [], []
            for f in fields:
                lo, hi, sg = mbl.sigma_midpoint(b, f, 1e-12)
                sig.append(sg)
                esc.append(max(abs(lo), abs(hi)))
            res = mbl.si_lanczos_batched(b, bt, fields, sig, nev, mmax=mmax, escale=esc,
                                         seed=first_seed)
            z = mbl.twist_expect_batched(b, bt, res.evecs)
            S_all = mbl.entanglement_entropy_batched(b, res.evecs)     # (R, nev), la = L/2
            rr, ss, zz = [], [], []
            for r in range(R):
                # the converged pairs (explicit residual within eig_tol * escale)
                idx = np.nonzero(res.resid[r] <= 1e-10 * esc[r])[0]
                k = len(idx)
                rr.append(mbl.spacing_ratio(res.evals[r][idx])[0] if k >= 3 else float("nan"))
                if k:
                    ss.append(float(np.mean(S_all[r][idx])))
                    zz.append(float(np.mean(np.abs(z[r][idx]) ** 2)))
                else:
                    ss.append(float("nan"))
                    zz.append(float("nan"))
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            per = [{"seed": first_seed + r, "sigma": float(sig[r]), "nconv": int(res.nconv[r]),
                    "r": float(rr[r]), "S": float(ss[r]), "z2": float(zz[r]),
                    "evals": [float(e) for e in res.evals[r]]} for r in range(R)]
            rr, ss, zz = np.array(rr), np.array(ss), np.array(zz)
            yield {"study": "scan", "L": L, "n": b.n, "h": h, "R": R, "nev": nev,
                   "nconv_min": int(res.nconv.min()), "seconds": round(dt, 1),
                   "r_mean": float(np.nanmean(rr)), "r_std": float(np.nanstd(rr)),
                   "r_goe": 0.5307, "r_poisson": 2 * math.log(2) - 1,
                   "S_mean": float(np.nanmean(ss)), "S_std": float(np.nanstd(ss)),
                   "S_rmt": float(0.5 * math.log(2) * L + 0.5 * math.log(0.5) - 0.25),
                   "z2_mean": float(np.nanmean(zz)), "z2_std": float(np.nanstd(zz)),
                   "two_over_n": 2.0 / b.n, "realizations": per}
        del bt


def main(argv=None):
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    ap = argparse.ArgumentParser()
    ap.add_argument("study", choices=["precond", "memory", "eig", "scan", "grad", "mixed"])
    ap.add_argument("--L", type=int, nargs="+", default=[12, 14, 16, 18])
    ap.add_argument("--h", type=float, nargs="+", default=[3.0, 4.0])
    ap.add_argument("--seeds", type=int, nargs="+", default=[0, 1])
    ap.add_argument("--mmax", type=int, default=130)
    ap.add_argument("--nev", type=int, default=4)
    ap.add_argument("--precision", default="fp64")
    ap.add_argument("--R", type=int, default=32)
    a = ap.parse_args(argv)
    if a.study == "precond":
        rows = precond_iterations(a.L, a.h, a.seeds)
    elif a.study == "memory":
        rows = memory_curve(a.L, a.mmax)
    elif a.study == "scan":
        rows = disorder_scan(a.L, a.h, a.R, a.nev, a.seeds[0])
    elif a.study == "mixed":
        rows = (r for L in a.L for s_ in a.seeds for r in mixed_study(L, a.h[0], s_, a.nev))
    elif a.study == "grad":
        rows = (r for L in a.L for r in grad_study(L, a.h[0], a.R, a.nev, a.seeds[0]))
    else:
        rows = (r for L in a.L for r in eigen_run(L, a.h[0], a.seeds[0], a.nev, a.precision))
    for r in rows:
        print(json.dumps(r), flush=True)


if __name__ == "__main__":
    main()
