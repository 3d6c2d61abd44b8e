"""Argument rejection at the C ABI with valid handles: every listed bad
argument returns MBL_ERR_ARG before anything is launched, leaves the output
buffers untouched and sets a message (mbl_last_error). Called through ctypes
directly, without the Python binding's own checks."""
import ctypes as C
import math
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

NAN, INF = float("nan"), float("inf")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def env(gpu):
    import torch
    mbl = gpu
    L = 10
    b = mbl.Basis(L)
    ws = mbl.Workspace(b, 20)
    n = b.n
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    y = torch.full((n,), 7.0, dtype=torch.float64, device="cuda")
    U = torch.full((4, n), 7.0, dtype=torch.float64, device="cuda")
    h = np.linspace(-1.0, 1.0, L)
    return dict(mbl=mbl, torch=torch, lib=mbl.lib, b=b, ws=ws, n=n, L=L, x=x, y=y, U=U, h=h)


def _h(a):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    return a, a.ctypes.data_as(C.POINTER(C.c_double))


def _expect_arg(env, st, untouched=()):
    mbl = env["mbl"]
    assert st == mbl.ERR_ARG, st
    assert mbl.lib.mbl_last_error().decode() != ""
    env["torch"].cuda.synchronize()
    for t in untouched:
        assert bool((t == 7.0).all()), "output written on an argument error"


def _ptr(t):
    return C.c_void_p(t.data_ptr())


def _bad_fields(env):
    L = env["L"]
    out = []
    for k, v in ((0, NAN), (3, INF), (L - 1, -INF)):
        f = env["h"].copy()
        f[k] = v
        out.append(f)
    return out


def test_apply_rejects_nonfinite_fields_and_shift(env):
    say("abi errors: apply_H")
    lib, b, x, y = env["lib"], env["b"], env["x"], env["y"]
    s = C.c_void_p(env["torch"].cuda.current_stream().cuda_stream)
    for f in _bad_fields(env):
        a, p = _h(f)
        _expect_arg(env, lib.mbl_apply_H(b.handle, p, 0.0, _ptr(x), _ptr(y), s), [y])
    a, p = _h(env["h"])
    for sg in (NAN, INF):
        _expect_arg(env, lib.mbl_apply_H(b.handle, p, sg, _ptr(x), _ptr(y), s), [y])
    _expect_arg(env, lib.mbl_apply_H(b.handle, p, 0.0, _ptr(y), _ptr(y), s), [y])
    for f in _bad_fields(env):
        a, p = _h(f)
        _expect_arg(env, lib.mbl_precond_apply(b.handle, p, 0.0, 0, _ptr(x), _ptr(y), s), [y])
    a, p = _h(env["h"])
    _expect_arg(env, lib.mbl_precond_apply(b.handle, p, 0.0, 3, _ptr(x), _ptr(y), s), [y])


@pytest.mark.parametrize("tol,kmax,sigma,prec,pc", [
    (0.0, 100, 0.0, 0, 0), (-1e-10, 100, 0.0, 0, 0), (NAN, 100, 0.0, 0, 0),
    (INF, 100, 0.0, 0, 0), (1e-10, 0, 0.0, 0, 0), (1e-10, -5, 0.0, 0, 0),
    (1e-10, 100, NAN, 0, 0), (1e-10, 100, INF, 0, 0), (1e-10, 100, 0.0, 2, 0),
    (1e-10, 100, 0.0, 0, -1)])
def test_minres_rejects(env, tol, kmax, sigma, prec, pc):
    say(f"abi errors: minres tol={tol} kmax={kmax} sigma={sigma} prec={prec} pc={pc}")
    lib, b, ws, x, y = env["lib"], env["b"], env["ws"], env["x"], env["y"]
    a, p = _h(env["h"])
    info = env["mbl"].MinresInfo()
    st = lib.mbl_minres_solve(b.handle, p, sigma, _ptr(x), _ptr(y), tol, kmax, prec, pc,
                              ws.handle, C.byref(info), None)
    _expect_arg(env, st, [y])


def test_minres_rejects_nonfinite_fields(env):
    lib, b, ws, x, y = env["lib"], env["b"], env["ws"], env["x"], env["y"]
    for f in _bad_fields(env):
        a, p = _h(f)
        st = lib.mbl_minres_solve(b.handle, p, 0.0, _ptr(x), _ptr(y), 1e-10, 100, 0, 0,
                                  ws.handle, None, None)
        _expect_arg(env, st, [y])


def _si(env, fields=None, sigma=0.0, nev=2, mmax=10, mtol=1e-10, mkmax=1000, etol=1e-10,
        ld=None, prec=0, pc=0):
    lib, b, ws, U = env["lib"], env["b"], env["ws"], env["U"]
    a, p = _h(env["h"] if fields is None else fields)
    ev = np.full(max(nev, 1), 7.0)
    res = np.full(max(nev, 1), 7.0)
    info = env["mbl"].SiInfo()
    st = lib.mbl_si_lanczos(b.handle, p, sigma, nev, mmax, mtol, mkmax, etol, 1e-5, 0.0, None,
                            1, prec, pc, ws.handle, ev.ctypes.data_as(C.POINTER(C.c_double)),
                            _ptr(U), env["n"] if ld is None else ld,
                            res.ctypes.data_as(C.POINTER(C.c_double)), C.byref(info), None)
    _expect_arg(env, st, [U])
    assert np.all(ev == 7.0) and np.all(res == 7.0)


def test_si_lanczos_rejects(env):
    say("abi errors: si_lanczos")
    n = env["n"]
    _si(env, nev=0)
    _si(env, nev=n + 1, mmax=20)          # nev > n
    _si(env, nev=5, mmax=4)               # mmax < nev
    _si(env, nev=2, mmax=21)              # mmax beyond the workspace
    _si(env, mkmax=0)                     # MINRES kmax < 1
    _si(env, mkmax=-3)
    _si(env, mtol=0.0)                    # MINRES tol <= 0
    _si(env, mtol=-1e-12)
    _si(env, mtol=NAN)
    _si(env, etol=0.0)                    # eigen tolerance <= 0
    _si(env, etol=NAN)
    _si(env, sigma=NAN)
    _si(env, sigma=INF)
    for f in _bad_fields(env):
        _si(env, fields=f)
    _si(env, ld=n - 1)
    _si(env, prec=5)
    _si(env, pc=7)


def test_eig_grad_rejects(env):
    say("abi errors: eig_grad")
    lib, b, ws, x = env["lib"], env["b"], env["ws"], env["x"]
    L = env["L"]
    dE, dz = np.full(L, 7.0), np.full(L, 7.0)
    dp = C.POINTER(C.c_double)
    lib.mbl_eig_grad.restype = C.c_int32
    lib.mbl_eig_grad.argtypes = [C.c_void_p, dp, C.c_double, C.c_void_p, C.c_double, C.c_int64,
                                 C.c_int, C.c_void_p, dp, dp, dp, C.c_void_p, C.c_void_p]
    a, p = _h(env["h"])
    for E, tol, kmax in ((NAN, 1e-10, 100), (INF, 1e-10, 100), (0.0, 0.0, 100),
                         (0.0, -1.0, 100), (0.0, NAN, 100), (0.0, 1e-10, 0)):
        st = lib.mbl_eig_grad(b.handle, p, E, _ptr(x), tol, kmax, 0, ws.handle,
                              dE.ctypes.data_as(dp), dz.ctypes.data_as(dp), None, None, None)
        _expect_arg(env, st)
        assert np.all(dE == 7.0) and np.all(dz == 7.0)
    for f in _bad_fields(env):
        a, p = _h(f)
        st = lib.mbl_eig_grad(b.handle, p, 0.0, _ptr(x), 1e-10, 100, 0, ws.handle,
                              dE.ctypes.data_as(dp), dz.ctypes.data_as(dp), None, None, None)
        _expect_arg(env, st)


def test_observable_and_sigma_calls_reject(env):
    say("abi errors: twist, residual, entropy, sigma")
    lib, b, U, n, L = env["lib"], env["b"], env["U"], env["n"], env["L"]
    dp = C.POINTER(C.c_double)
    z = np.full(8, 7.0)
    _expect_arg(env, lib.mbl_twist_expect(b.handle, _ptr(U), n, 0, z.ctypes.data_as(dp), None))
    _expect_arg(env, lib.mbl_twist_expect(b.handle, _ptr(U), n - 1, 1, z.ctypes.data_as(dp), None))
    assert np.all(z == 7.0)
    S = np.full(4, 7.0)
    for la in (0, L, -1):
        _expect_arg(env, lib.mbl_entanglement_entropy(b.handle, _ptr(U), n, 1, la,
                                                      S.ctypes.data_as(dp), None))
    assert np.all(S == 7.0)
    E = np.zeros(2)
    r = np.full(2, 7.0)
    for f in _bad_fields(env):
        a, p = _h(f)
        _expect_arg(env, lib.mbl_eig_residual(b.handle, p, E.ctypes.data_as(dp), _ptr(U), n, 2,
                                              r.ctypes.data_as(dp), None))
        lo, hi, sg = C.c_double(7.0), C.c_double(7.0), C.c_double(7.0)
        _expect_arg(env, lib.mbl_sigma_midpoint(b.handle, p, 1e-10, 0, C.byref(lo), C.byref(hi),
                                                C.byref(sg), None))
        assert lo.value == hi.value == sg.value == 7.0
    a, p = _h(env["h"])
    lo, hi, sg = C.c_double(7.0), C.c_double(7.0), C.c_double(7.0)
    for rt in (0.0, -1e-3, NAN):
        _expect_arg(env, lib.mbl_sigma_midpoint(b.handle, p, rt, 0, C.byref(lo), C.byref(hi),
                                                C.byref(sg), None))
    assert np.all(r == 7.0)


def test_batched_calls_reject(env):
    say("abi errors: batched")
    mbl, lib, torch = env["mbl"], env["lib"], env["torch"]
    b = mbl.Basis(12)
    vp = C.c_void_p
    lib.mbl_batch_create.restype = C.c_int32
    lib.mbl_batch_create.argtypes = [vp, C.c_int, C.c_int, C.c_int, C.POINTER(vp)]
    out = vp()
    for R in (0, 1, 3, 6, 64):
        _expect_arg(env, lib.mbl_batch_create(b.handle, R, 0, 0, C.byref(out)))
    _expect_arg(env, lib.mbl_batch_create(b.handle, 4, 1001, 1, C.byref(out)))
    _expect_arg(env, lib.mbl_batch_create(b.handle, 4, 10, 11, C.byref(out)))
    R = 4
    bt = mbl.Batch(b, R, mmax=12, nevmax=2)
    n = b.n
    X = torch.ones((n, R), dtype=torch.float64, device="cuda")
    Y = torch.full((n, R), 7.0, dtype=torch.float64, device="cuda")
    fields = np.tile(np.linspace(-1, 1, 12), (R, 1))
    dp = C.POINTER(C.c_double)
    lib.mbl_minres_solve_batched.restype = C.c_int32
    lib.mbl_minres_solve_batched.argtypes = [vp, vp, dp, dp, vp, vp, C.c_double, C.c_int64, C.c_int,
                                             C.c_int, vp, vp, vp]
    sig = np.zeros(R)
    for tol, kmax in ((0.0, 10), (-1.0, 10), (NAN, 10), (1e-10, 0)):
        a, p = _h(fields)
        st = lib.mbl_minres_solve_batched(b.handle, bt.handle, p, sig.ctypes.data_as(dp), _ptr(X),
                                          _ptr(Y), tol, kmax, 0, 0, None, None, None)
        _expect_arg(env, st, [Y])
    bad = fields.copy()
    bad[2, 5] = NAN
    a, p = _h(bad)
    st = lib.mbl_minres_solve_batched(b.handle, bt.handle, p, sig.ctypes.data_as(dp), _ptr(X),
                                      _ptr(Y), 1e-10, 10, 0, 0, None, None, None)
    _expect_arg(env, st, [Y])
    a, p = _h(fields)
    sg = sig.copy()
    sg[1] = INF
    st = lib.mbl_minres_solve_batched(b.handle, bt.handle, p, sg.ctypes.data_as(dp), _ptr(X),
                                      _ptr(Y), 1e-10, 10, 0, 0, None, None, None)
    _expect_arg(env, st, [Y])
    # a batch workspace of another basis
    b2 = mbl.Basis(12)
    st = lib.mbl_minres_solve_batched(b2.handle, bt.handle, p, sig.ctypes.data_as(dp), _ptr(X),
                                      _ptr(Y), 1e-10, 10, 0, 0, None, None, None)
    _expect_arg(env, st, [Y])
    assert math.isfinite(float(X.sum()))
