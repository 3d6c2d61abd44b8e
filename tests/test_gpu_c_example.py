"""The C ABI from a plain C99 program (paper_2203_09732_amd/examples/
mbl_example.c, built by build()): its products, sigma, MINRES solution,
eigenpairs and twist overlaps against the oracle."""
import os
import subprocess
import sys

import numpy as np
import pytest

from oracle import lanczos, minres, model, twist
from workloads import disorder_fields

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EXE = os.path.join(ROOT, "paper_2203_09732_amd", "mbl_example")


def test_c_program_against_oracle(gpu):
    if not os.path.exists(EXE):
        pytest.skip("paper_2203_09732_amd/mbl_example is built by build(); not built here")
    L = 12
    h = disorder_fields(L, 3.0, 4)
    print(f"running {EXE} L={L}", flush=True)
    sys.stdout.flush()
    r = subprocess.run([EXE, str(L)], input=" ".join(repr(float(v)) for v in h),
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    out = {}
    for line in r.stdout.splitlines():
        key, *vals = line.split()
        out[key] = vals
    n = int(out["n"][0])
    H = model.hamiltonian_csr(L, h)
    assert n == H.shape[0]
    x = np.sin(np.arange(1, n + 1, dtype=np.float64))
    y = np.array(out["apply"], dtype=float)
    yref = H @ x - 0.25 * x
    assert np.abs(y - yref).max() <= 1e-13 * np.abs(yref).max()
    w, V = np.linalg.eigh(H.toarray())
    emin, emax, sigma = map(float, out["sigma"])
    assert abs(emin - w[0]) <= 1e-10 * abs(w[0]) and abs(emax - w[-1]) <= 1e-10 * abs(w[-1])
    st, iters = int(out["minres"][0]), int(out["minres"][1])
    assert st == 0 and iters > 0
    v = np.array(out["solution"], dtype=float)
    vref = minres.solve_dense(H.toarray(), sigma, x)
    assert np.linalg.norm(v - vref) <= 1e-8 * np.linalg.norm(vref)
    assert int(out["lanczos"][0]) == 0 and int(out["lanczos"][2]) == 4
    E = np.array(out["evals"], dtype=float)
    Eref, Uref = lanczos.eigenpairs_dense(H.toarray(), sigma, 4)
    assert np.all(np.abs(E - Eref) <= 1e-10 * np.maximum(np.abs(Eref), 1))
    resid = np.array(out["resid"], dtype=float)
    assert resid.max() <= 1e-9
    # |z - z_ref| <= 2 ||u - u_ref|| <= 2 resid / gap
    gaps = np.array([np.min(np.abs(np.delete(w, np.argmin(np.abs(w - e))) - e)) for e in E])
    z = np.array(out["z"], dtype=float)
    zref = twist.twist_overlap(L, Uref)
    assert np.all(np.abs((z[0::2] + 1j * z[1::2]) - zref) <= 2 * resid / gaps + 1e-12)
