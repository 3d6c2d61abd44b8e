"""Writes the stored expected values under tests/golden/ from the CPU oracle.

Only ``oracle`` and the seeded input generators are used. Run from the
repository root:

    python tests/golden/make_golden.py            (the L = 14 dense reference)
    python tests/golden/make_golden.py --si 16    (sparse shift-invert, L = 16)
    python tests/golden/make_golden.py --si 18    (the same at L = 18, ~20 min)
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import lanczos, model, twist  # noqa: E402
from workloads import disorder_fields  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def plain(L, h, seed, nev):
    f = disorder_fields(L, h, seed)
    H = model.hamiltonian_dense(L, f)
    w = np.linalg.eigvalsh(H)
    sigma = 0.5 * (w[0] + w[-1])
    E, V = lanczos.eigenpairs_dense(H, sigma, nev)
    z = twist.twist_overlap(L, V)
    idx = np.searchsorted(w, E)
    gaps = [float(min(abs(w[i] - w[i - 1]) if i > 0 else np.inf,
                      abs(w[i + 1] - w[i]) if i + 1 < len(w) else np.inf)) for i in idx]
    return {
        "L": L, "h": h, "seed": seed, "nev": nev,
        "fields": f.tolist(),
        "E_min": float(w[0]), "E_max": float(w[-1]), "sigma": float(sigma),
        "evals": E.tolist(), "gaps": gaps,
        "z_re": np.real(z).tolist(), "z_im": np.imag(z).tolist(),
        "source": "oracle dense eigensolver (oracle.lanczos.eigenpairs_dense), twist by oracle.twist",
    }


def shift_invert(L, h, seed, nev, window):
    """sigma = (E_min + E_max) / 2 from the oracle's extremal eigenvalues, the
    `window` eigenvalues nearest sigma from the oracle's sparse shift-invert
    solver (for the gaps of the selected pairs), the nev nearest of them with
    the twist overlaps of their eigenvectors."""
    f = disorder_fields(L, h, seed)
    H = model.hamiltonian_csr(L, f)
    emin, emax = lanczos.extremal_eigenvalues(H)
    sigma = 0.5 * (emin + emax)
    w, V = lanczos.eigenpairs_shift_invert_sparse(H, sigma, window)
    sel = lanczos.select_nearest(w, sigma, nev)
    E, U = w[sel], V[:, sel]
    z = twist.twist_overlap(L, U)
    res = lanczos.eigen_residuals(H, E, U)
    return {
        "L": L, "h": h, "seed": seed, "nev": nev,
        "fields": f.tolist(),
        "E_min": float(emin), "E_max": float(emax), "sigma": float(sigma),
        "evals": E.tolist(), "window": w.tolist(),
        "z_re": np.real(z).tolist(), "z_im": np.imag(z).tolist(),
        "oracle_residuals": res.tolist(),
        "source": "oracle sparse shift-invert (oracle.lanczos.eigenpairs_shift_invert_sparse, "
                  f"{window} eigenvalues nearest sigma), extremes by "
                  "oracle.lanczos.extremal_eigenvalues, twist by oracle.twist",
    }


if __name__ == "__main__":
    if "--si" in sys.argv:
        L = int(sys.argv[sys.argv.index("--si") + 1])
        out = shift_invert(L, 3.0, 0, 6, 12)
        name = f"si_L{L}_h3_seed0.json"
        with open(os.path.join(HERE, name), "w") as fh:
            json.dump(out, fh, indent=1)
        print("wrote", name, out["sigma"], out["evals"])
        sys.exit(0)
    out = plain(14, 3.0, 0, 10)
    with open(os.path.join(HERE, "plain_L14_h3_seed0.json"), "w") as fh:
        json.dump(out, fh, indent=1)
    print("wrote plain_L14_h3_seed0.json", out["sigma"], out["evals"][:3])
