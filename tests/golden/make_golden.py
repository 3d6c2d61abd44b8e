"""Writes the stored expected values under tests/golden/ from the CPU oracle.

Only ``oracle`` and the seeded input generators are used. Run from the
repository root:  python tests/golden/make_golden.py
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


if __name__ == "__main__":
    out = plain(14, 3.0, 0, 10)
    with open(os.path.join(HERE, "plain_L14_h3_seed0.json"), "w") as fh:
        json.dump(out, fh, indent=1)
    print("wrote plain_L14_h3_seed0.json", out["sigma"], out["evals"][:3])
