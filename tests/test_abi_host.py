"""C-ABI library checks that need no GPU: it loads, exports every symbol the
header declares, rejects bad arguments before touching a device, and its
host-only tridiagonal eigensolver agrees with LAPACK."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    text = open(os.path.join(ROOT, "include", "mbl.h")).read()
    return sorted(set(re.findall(r"\b(mbl_[A-Za-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def mbl():
    import paper_2203_09732_amd as m
    return m


def test_every_declared_symbol_is_exported(mbl):
    syms = _declared_symbols()
    assert len(syms) >= 20
    for s in syms:
        assert hasattr(mbl.lib, s), s


def test_version(mbl):
    assert "gfx950" in mbl.version()


@pytest.mark.parametrize("L", [3, 5, 2, 0, 34, -4])
def test_build_basis_rejects_bad_L(mbl, L):
    h = C.c_void_p()
    st = mbl.lib.mbl_build_basis(L, 0, None, C.byref(h))
    assert st == mbl.ERR_ARG
    assert "L must be even" in mbl.lib.mbl_last_error().decode()


@pytest.mark.parametrize("L,lo", [(8, 8), (8, -1), (20, 14), (30, 15)])
def test_build_basis_rejects_bad_split(mbl, L, lo):
    h = C.c_void_p()
    assert mbl.lib.mbl_build_basis(L, lo, None, C.byref(h)) == mbl.ERR_ARG


def test_null_handles_rejected(mbl):
    hh = (C.c_double * 4)()
    assert mbl.lib.mbl_apply_H(None, hh, 0.0, None, None, None) == mbl.ERR_ARG
    assert mbl.lib.mbl_precond_apply(None, hh, 0.0, 0, None, None, None) == mbl.ERR_ARG
    assert mbl.lib.mbl_minres_solve(None, hh, 0.0, None, None, 1e-12, 10, 0, 0, None, None,
                                    None) == mbl.ERR_ARG
    assert mbl.lib.mbl_twist_expect(None, None, 0, 1, None, None) == mbl.ERR_ARG
    n = C.c_int64()
    assert mbl.lib.mbl_basis_dim(None, C.byref(n)) == mbl.ERR_ARG
    out = C.c_double()
    assert mbl.lib.mbl_dot(-1, None, None, C.byref(out), None) == mbl.ERR_ARG
    assert mbl.lib.mbl_dot(0, None, None, C.byref(out), None) == mbl.OK and out.value == 0.0


def _problem(mbl, L, nev, h=None, sigma=float("nan")):
    """One mbl_problem with host arrays kept alive on the returned object and
    a non-NULL fake device pointer (never touched: these calls fail argument
    checks before any device work)."""
    p = mbl.Problem()
    hh = np.zeros(L) if h is None else np.asarray(h, dtype=np.float64)
    ev = np.zeros(max(nev, 1))
    p._keep = (hh, ev)
    p.L, p.nev = L, nev
    p.h_host = hh.ctypes.data_as(C.POINTER(C.c_double))
    p.sigma, p.escale = sigma, 0.0
    p.evecs_dev = 0x1000
    p.evals_host = ev.ctypes.data_as(C.POINTER(C.c_double))
    return p


@pytest.mark.parametrize("case", ["odd L", "L too large", "nev 0", "nev > 32", "nan field",
                                  "inf sigma", "nev > n"])
def test_problem_array_rejects_bad_problems_on_the_host(mbl, case):
    L, nev, h, sigma = 10, 2, None, float("nan")
    if case == "odd L":
        L = 11
    elif case == "L too large":
        L = 34
    elif case == "nev 0":
        nev = 0
    elif case == "nev > 32":
        nev = 33
    elif case == "nan field":
        h = np.full(10, np.nan)
    elif case == "inf sigma":
        sigma = float("inf")
    elif case == "nev > n":
        L, nev = 4, 7          # C(4, 2) = 6 states
    arr = (mbl.Problem * 1)(_problem(mbl, L, nev, h, sigma))
    st = mbl.lib.mbl_si_lanczos_problems(arr, 1, 0, 1e-12, 1000, 1e-10, 1e-5, 0, 0, None)
    assert st == mbl.ERR_ARG, (case, mbl.lib.mbl_last_error().decode())


def test_problem_array_rejects_bad_call_arguments_on_the_host(mbl, monkeypatch):
    arr = (mbl.Problem * 1)(_problem(mbl, 10, 2))
    call = mbl.lib.mbl_si_lanczos_problems
    assert call(None, 1, 0, 1e-12, 1000, 1e-10, 1e-5, 0, 0, None) == mbl.ERR_ARG
    assert call(arr, 0, 0, 1e-12, 1000, 1e-10, 1e-5, 0, 0, None) == mbl.ERR_ARG
    assert call(arr, 1, 129, 1e-12, 1000, 1e-10, 1e-5, 0, 0, None) == mbl.ERR_ARG   # mmax
    assert call(arr, 1, 0, 0.0, 1000, 1e-10, 1e-5, 0, 0, None) == mbl.ERR_ARG       # minres_tol
    assert call(arr, 1, 0, 1e-12, 0, 1e-10, 1e-5, 0, 0, None) == mbl.ERR_ARG        # kmax
    assert call(arr, 1, 0, 1e-12, 1000, -1.0, 1e-5, 0, 0, None) == mbl.ERR_ARG      # eig_tol
    assert call(arr, 1, 0, 1e-12, 1000, 1e-10, 1e-5, 0, 3, None) == mbl.ERR_ARG     # precond
    for bad in ("7", "18", "8", "11"):
        monkeypatch.setenv("MBL_PERSISTENT_MAX_L", bad)
        assert call(arr, 1, 0, 1e-12, 1000, 1e-10, 1e-5, 0, 0, None) == mbl.ERR_ARG
        assert "MBL_PERSISTENT_MAX_L" in mbl.lib.mbl_last_error().decode()


def test_batch_schedule_rejects_null_handle(mbl):
    assert mbl.lib.mbl_batch_set_schedule(None, 0, 0, 0) == mbl.ERR_ARG


@pytest.mark.parametrize("k,seed", [(1, 0), (2, 1), (7, 2), (60, 3), (250, 4)])
def test_tridiag_eig_matches_lapack(mbl, k, seed):
    rng = np.random.default_rng(seed)
    a = rng.standard_normal(k)
    b = rng.uniform(0.1, 2.0, max(k - 1, 0))
    w, V = mbl.tridiag_eig(a, b)
    T = np.diag(a) + (np.diag(b, 1) + np.diag(b, -1) if k > 1 else 0)
    wr = np.linalg.eigvalsh(T)
    assert np.allclose(w, wr, atol=1e-12 * max(1, np.abs(wr).max()))
    assert np.allclose(T @ V, V * w[None, :], atol=1e-11)
    assert np.allclose(V.T @ V, np.eye(k), atol=1e-12)


def test_tridiag_eig_clustered_and_split():
    import paper_2203_09732_amd as mbl
    # Wilkinson W21+: nearly degenerate pairs; and a split (zero off-diagonal)
    a = np.abs(np.arange(-10, 11)).astype(float)
    b = np.ones(20)
    b[7] = 0.0
    w, V = mbl.tridiag_eig(a, b)
    T = np.diag(a) + np.diag(b, 1) + np.diag(b, -1)
    assert np.allclose(w, np.linalg.eigvalsh(T), atol=1e-12)
    assert np.allclose(T @ V, V * w[None, :], atol=1e-11)


@pytest.mark.parametrize("scale", [1e-150, 1.0, 1e150])
def test_tridiag_eig_graded_and_scaled(mbl, scale):
    """A graded matrix (entries falling by 10^-0.5 per row) and W21+ at
    scales far from 1: eigenvalues to 1e-12 of the largest, eigenvectors
    orthonormal and with residuals to 1e-11 relative."""
    k = 40
    a = scale * 10.0 ** (-0.5 * np.arange(k))
    b = scale * 0.3 * 10.0 ** (-0.5 * np.arange(k - 1) - 0.25)
    for aa, bb in ((a, b), (scale * np.abs(np.arange(-10, 11)).astype(float), scale * np.ones(20))):
        w, V = mbl.tridiag_eig(aa, bb)
        T = np.diag(aa) + np.diag(bb, 1) + np.diag(bb, -1)
        wr = np.linalg.eigvalsh(T)
        top = np.abs(wr).max()
        assert np.all(np.abs(w - wr) <= 1e-12 * top)
        assert np.abs(T @ V - V * w[None, :]).max() <= 1e-11 * top
        assert np.allclose(V.T @ V, np.eye(len(aa)), atol=1e-12)


def test_single_hip_runtime_in_process():
    """The binding loads torch's HIP runtime first, so libmbl.so resolves its
    libamdhip64.so.7 dependency to it: one runtime serves torch's streams and
    allocations and the library's launches."""
    import subprocess
    import sys
    code = ("import sys; sys.path.insert(0, %r); import paper_2203_09732_amd; "
            "m = open('/proc/self/maps').read(); "
            "print(len(set(l.split()[-1] for l in m.splitlines() if 'amdhip64' in l)))") % ROOT
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip().splitlines()[-1] == "1"


def test_spacing_ratio_matches_oracle(mbl):
    """Host-only level-spacing ratio (Sec. IV) against the oracle's."""
    from oracle import observables
    rng = np.random.default_rng(3)
    for n in (3, 4, 17, 500):
        E = rng.standard_normal(n)
        mean, r = mbl.spacing_ratio(E)
        want = observables.spacing_ratios(E)
        assert np.allclose(r, want, rtol=0, atol=1e-15)
        assert abs(mean - observables.mean_spacing_ratio(E)) <= 1e-15
    mean, r = mbl.spacing_ratio([0.0, 1.0, 1.0, 1.0, 2.0])
    assert np.isnan(r[1]) and r[0] == 0.0 and r[2] == 0.0 and mean == 0.0
    mean, r = mbl.spacing_ratio([2.0, 2.0, 2.0])
    assert np.isnan(mean)


def test_spacing_ratio_rejects_bad_input(mbl):
    for E in ([1.0, 2.0], [0.0, np.nan, 1.0, 2.0], [0.0, np.inf, 1.0]):
        with pytest.raises(mbl.MblError):
            mbl.spacing_ratio(E)


def _graded_psd(rng, m, c, r, decay, zero_row):
    U, _ = np.linalg.qr(rng.standard_normal((m, m)))
    V, _ = np.linalg.qr(rng.standard_normal((c, c)))
    s = np.zeros(m)
    s[:r] = decay ** np.arange(r)
    X = (U * s) @ V[:m, :]
    if zero_row is not None:
        X[zero_row, :] = 0.0
    return X @ X.T


def test_symmetric_eigenvalues_graded_and_rank_deficient(mbl):
    """The host routine behind the entanglement entropy, on the matrices its
    Schmidt blocks produce: Gram matrices of rank r <= m with singular values
    decaying geometrically, zero rows, rank one (all entries equal), and a
    column far below the trailing block. Against LAPACK, to 2e-14 ||A||."""
    rng = np.random.default_rng(7)
    cases = []
    for t in range(150):
        m = int(rng.integers(1, 90))
        c = int(rng.integers(m, 2 * m + 5))
        r = int(rng.integers(1, m + 1))
        cases.append(_graded_psd(rng, m, c, r, 10.0 ** (-rng.uniform(0, 3)),
                                 int(rng.integers(0, m)) if t % 7 == 0 else None))
    cases.append(np.full((70, 70), 437.5))
    B = rng.standard_normal((12, 12))
    B = B @ B.T
    B[1:, 0] = B[0, 1:] = 1e-160 * rng.standard_normal(11)
    cases.append(B)
    for A in cases:
        w = mbl.symmetric_eigenvalues(A)
        ref = np.linalg.eigvalsh(A)
        assert np.abs(w - ref).max() <= 2e-14 * max(np.abs(ref).max(), 1e-300)


def test_symmetric_eigenvalues_rejects_bad_input(mbl):
    with pytest.raises(mbl.MblError):
        mbl.symmetric_eigenvalues(np.array([[1.0, np.nan], [np.nan, 1.0]]))
