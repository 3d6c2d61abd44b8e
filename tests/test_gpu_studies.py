"""The studies beyond the hot path, checked at small size.

* Disorder scan (Sec. IV): per realization, the mean level-spacing ratio,
  the mean half-chain entanglement entropy and the mean |z|^2 over the pairs
  the batched eigen-run returns, against the oracle's dense eigenpairs of the
  same fields (the nev nearest the spectral midpoint), L = 12 and 14, h = 1
  and 4, four realizations each.
  Bars: the ratio depends on the eigenvalues only (1e-10 relative each, gaps
  >= 1e-3 here): 1e-7. S and |z|^2 of a vector within sin(theta) <= 1e-5 of
  the exact eigenvector (residual <= 1e-10 ||H||, gap test 1e-5): by
  Fannes-Audenaert |dS| <= T ln(d - 1) + H(T) with T <= sin(theta), so 3e-4
  covers it; |d|z|^2| <= 4 sin(theta) <= 4e-5.
* Memory against L (Sec. IV A): the device memory a workspace takes,
  measured as the drop of the device's free memory across its creation, is
  at least the linear model 8 n (13 + mmax + 1) and exceeds it by at most the
  runtime's allocation rounding.
"""
import sys

import numpy as np
import pytest

from oracle import lanczos, model, observables, twist
from workloads import disorder_fields

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_disorder_scan_matches_oracle(gpu):
    from paper_2203_09732_amd import studies
    R, nev = 4, 6
    for row in studies.disorder_scan([12, 14], [1.0, 4.0], R=R, nev=nev, first_seed=0):
        L, h = row["L"], row["h"]
        say(f"scan L={L} h={h}: r={row['r_mean']:.4f} S={row['S_mean']:.4f} z2={row['z2_mean']:.4f}")
        assert row["nconv_min"] == nev
        for rec in row["realizations"]:
            f = disorder_fields(L, h, rec["seed"])
            H = model.hamiltonian_dense(L, f)
            w = np.linalg.eigvalsh(H)
            sigma = 0.5 * (w[0] + w[-1])
            assert abs(rec["sigma"] - sigma) <= 1e-10 * max(abs(w[0]), abs(w[-1]))
            E, V = lanczos.eigenpairs_dense(H, sigma, nev)
            assert np.all(np.abs(np.array(rec["evals"]) - E) / np.maximum(np.abs(E), 1) <= 1e-10)
            r_ref = observables.mean_spacing_ratio(E)
            S_ref = np.mean([observables.entanglement_entropy(L, V[:, t]) for t in range(nev)])
            z2_ref = np.mean(np.abs(twist.twist_overlap(L, V)) ** 2)
            assert abs(rec["r"] - r_ref) <= 1e-7, (rec["r"], r_ref)
            assert abs(rec["S"] - S_ref) <= 3e-4, (rec["S"], S_ref)
            assert abs(rec["z2"] - z2_ref) <= 4e-5, (rec["z2"], z2_ref)
        # the row's statistics are those of its realizations
        assert abs(row["r_mean"] - np.mean([x["r"] for x in row["realizations"]])) <= 1e-15
        assert abs(row["S_mean"] - np.mean([x["S"] for x in row["realizations"]])) <= 1e-15


def test_memory_curve_measured_against_linear_model(gpu):
    from paper_2203_09732_amd import studies
    mmax = 40
    for row in studies.memory_curve([14, 16, 18, 20, 22], mmax=mmax):
        model_b = row["model_8n(13+mmax+1)"]
        taken = row["device_bytes_taken"]
        say(f"memory L={row['L']}: taken {taken / 1e6:.1f} MB, model {model_b / 1e6:.1f} MB, "
            f"library count {row['workspace_bytes'] / 1e6:.1f} MB")
        assert taken >= model_b
        # per-allocation rounding (about 20 buffers) and the small fixed part
        assert taken <= 1.1 * model_b + 64 * 2**20


def test_grad_study_matches_oracle(gpu):
    """The gradient study's path (problem-array eigenpairs, then eig_grad per
    pair) at L = 10, 3 realizations, 2 pairs: dE/dh against the oracle's
    Hellmann-Feynman -<S^z_j> of its own dense eigenvector and d|z|^2/dh
    against the oracle's perturbation sum, at the bars of the adjoint tests;
    the sum rules the study reports."""
    from oracle import adjoint, model
    from paper_2203_09732_amd import studies
    from workloads import disorder_fields
    L, h, R, nev = 10, 3.0, 3, 2
    rows = list(studies.grad_study(L, h, R=R, nev=nev, first_seed=50))
    summary = rows[-1]
    assert summary["study"] == "grad_summary" and summary["converged_pairs"] == R * nev
    assert summary["max_abs_sum_dE"] <= 1e-11 and summary["max_rel_sum_dz2"] <= 1e-8
    for row in rows[:-1]:
        f = disorder_fields(L, h, row["seed"])
        w = np.linalg.eigvalsh(model.hamiltonian_dense(L, f))
        for q in row["pairs"]:
            k = int(np.argmin(np.abs(w - q["E"])))
            _, psi_ref, dpsi = adjoint.eigvec_derivatives(L, f, k)
            assert np.abs(np.array(q["dE"]) - adjoint.hellmann_feynman(L, psi_ref)).max() <= 5e-10
            dz2_ref = adjoint.dz2_dh(L, psi_ref, dpsi)
            assert np.abs(np.array(q["dz2"]) - dz2_ref).max() <= 1e-7 * max(1.0, np.abs(dz2_ref).max())


def test_mixed_study_reports_agreement(gpu):
    """The mixed-precision study at L = 12: both forms converge every pair
    and agree to the eigenpair bars (the FP32-inner form itself is checked
    against stored oracle references at L = 16 and 18 elsewhere)."""
    from paper_2203_09732_amd import studies
    (row,) = list(studies.mixed_study(12, 3.5, 3, 4))
    assert row["fp64"]["nconv"] == 4 and row["fp32_inner"]["nconv"] == 4
    assert row["max_rel_dE"] <= 1e-10 and row["max_overlap_deficit"] <= 1e-10
    assert row["max_dz"] <= 2 * np.sqrt(2 * 1e-10)   # |dz| <= 2 ||du||
    assert row["fp64"]["max_rel_resid"] <= 1e-10 and row["fp32_inner"]["max_rel_resid"] <= 1e-10
