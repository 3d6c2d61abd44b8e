"""Python binding of libmbl.so, the gfx950 library for nested shift-invert
diagonalization of the random-field Heisenberg chain (arXiv:2203.09732).

This module only marshals arguments: device buffers are torch tensors on the
current HIP device (``tensor.data_ptr()``), streams are
``torch.cuda.current_stream().cuda_stream``, and every step of the method
runs in the library's kernels. Importing fails if libmbl.so has not been
built (``python paper_2203_09732_amd/build.py``).
"""
from __future__ import annotations

import ctypes as C
import math
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmbl.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build it with `python paper_2203_09732_amd/build.py` "
        "(hipcc, gfx950). There is no fallback implementation.")

# One HIP runtime per process: torch ships its own libamdhip64 (same SONAME,
# libamdhip64.so.7, but NEEDED by torch under the bare name). Loading torch
# first makes the dynamic loader resolve libmbl's dependency to the runtime
# torch already mapped, so torch's streams and allocations and this library's
# launches go through one runtime. Loading libmbl first would map a second
# runtime beside torch's.
import torch as _torch  # noqa: E402,F401

lib = C.CDLL(LIB_PATH)

OK, ERR_ARG, ERR_NOMEM, ERR_HIP, ERR_NUMERIC = 0, -1, -2, -3, -4
WARN_NOCONV, WARN_BREAKDOWN = 1, 2
FP64, FP32_INNER = 0, 1
PRECOND = {"row": 0, "jacobi": 1, "id": 2}
PRECISION = {"fp64": FP64, "fp32_inner": FP32_INNER}

_vp, _dp, _i32, _i64, _u64, _d = C.c_void_p, C.POINTER(C.c_double), C.c_int32, C.c_int64, C.c_uint64, C.c_double


class MinresInfo(C.Structure):
    _fields_ = [("iters", C.c_int64), ("restarts", C.c_int32), ("phi", C.c_double),
                ("true_res", C.c_double)]


class SiInfo(C.Structure):
    _fields_ = [("steps", C.c_int32), ("nconv", C.c_int32), ("minres_iters", C.c_int64),
                ("max_rel_resid", C.c_double), ("seconds", C.c_double)]


def _sig(name, res, args):
    f = getattr(lib, name)
    f.restype = res
    f.argtypes = args
    return f


_sig("mbl_last_error", C.c_char_p, [])
_sig("mbl_version", C.c_char_p, [])
_sig("mbl_build_basis", _i32, [C.c_int, C.c_int, _vp, C.POINTER(_vp)])
_sig("mbl_basis_free", None, [_vp])
_sig("mbl_basis_dim", _i32, [_vp, C.POINTER(C.c_int64)])
_sig("mbl_basis_lo_bits", _i32, [_vp, C.POINTER(C.c_int)])
_sig("mbl_basis_states", _i32, [_vp, _vp, _vp])
_sig("mbl_basis_rank", _i32, [_vp, _vp, _i64, _vp, _vp])
_sig("mbl_workspace_create", _i32, [_vp, C.c_int, C.c_int, C.POINTER(_vp)])
_sig("mbl_workspace_free", None, [_vp])
_sig("mbl_workspace_bytes", _i32, [_vp, C.POINTER(C.c_int64)])
_sig("mbl_apply_H", _i32, [_vp, _dp, _d, _vp, _vp, _vp])
_sig("mbl_apply_H_f32", _i32, [_vp, _dp, _d, _vp, _vp, _vp])
_sig("mbl_precond_apply", _i32, [_vp, _dp, _d, C.c_int, _vp, _vp, _vp])
_sig("mbl_minres_solve", _i32, [_vp, _dp, _d, _vp, _vp, _d, _i64, C.c_int, C.c_int, _vp,
                                C.POINTER(MinresInfo), _vp])
_sig("mbl_si_lanczos", _i32, [_vp, _dp, _d, C.c_int, C.c_int, _d, _i64, _d, _d, _d, _vp, _u64,
                              C.c_int, C.c_int, _vp, _dp, _vp, _i64, _dp, C.POINTER(SiInfo), _vp])
_sig("mbl_twist_expect", _i32, [_vp, _vp, _i64, C.c_int, _dp, _vp])
_sig("mbl_twist_expect_noalloc", _i32, [_vp, _vp, _i64, C.c_int, _dp, _vp])
_sig("mbl_entanglement_entropy", _i32, [_vp, _vp, _i64, C.c_int, C.c_int, _dp, _vp])
_sig("mbl_spacing_ratio", _i32, [C.c_int, _dp, _dp, _dp])
_sig("mbl_symmetric_eigenvalues", _i32, [C.c_int, _dp, _dp])
_sig("mbl_entanglement_entropy_interleaved", _i32, [_vp, _vp, C.c_int, C.c_int, C.c_int, _dp, _vp])
_sig("mbl_eig_residual", _i32, [_vp, _dp, _dp, _vp, _i64, C.c_int, _dp, _vp])
_sig("mbl_sigma_midpoint", _i32, [_vp, _dp, _d, C.c_int, _dp, _dp, _dp, _vp])
_sig("mbl_dot", _i32, [_i64, _vp, _vp, _dp, _vp])
_sig("mbl_tridiag_eig", _i32, [C.c_int, _dp, _dp, _dp, _dp])


class MblError(RuntimeError):
    def __init__(self, status, where):
        msg = lib.mbl_last_error().decode()
        super().__init__(f"{where}: status {status}: {msg}")
        self.status = status


def _check(st, where, warn_ok=True):
    if st < 0 or (st > 0 and not warn_ok):
        raise MblError(st, where)
    return st


def version() -> str:
    return lib.mbl_version().decode()


def _f64(a):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    return a, a.ctypes.data_as(_dp)


def _stream(stream=None):
    if stream is not None:
        return C.c_void_p(stream)
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr())


def _need_cuda(t, dtype, n=None, name="tensor"):
    import torch
    if not t.is_cuda or t.dtype != dtype or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous {dtype} tensor on the GPU")
    if n is not None and t.numel() < n:
        raise ValueError(f"{name} has {t.numel()} elements, need {n}")
    return torch


class Basis:
    """Sector basis of the S^z = 0 sector of an L-site ring (dim C(L, L/2))."""

    def __init__(self, L: int, lo_bits: int = 0, stream=None):
        h = C.c_void_p()
        _check(lib.mbl_build_basis(int(L), int(lo_bits), _stream(stream), C.byref(h)),
               "mbl_build_basis", warn_ok=False)
        self._h = h
        self.L = int(L)
        n = C.c_int64()
        _check(lib.mbl_basis_dim(h, C.byref(n)), "mbl_basis_dim")
        self.n = int(n.value)
        lb = C.c_int()
        _check(lib.mbl_basis_lo_bits(h, C.byref(lb)), "mbl_basis_lo_bits")
        self.lo_bits = int(lb.value)

    @property
    def handle(self):
        return self._h

    def __del__(self):
        if getattr(self, "_h", None) and lib is not None:
            try:
                lib.mbl_basis_free(self._h)
            except Exception:   # interpreter shutdown
                pass
            self._h = None

    def states(self, stream=None):
        import torch
        out = torch.empty(self.n, dtype=torch.int32, device="cuda")
        _check(lib.mbl_basis_states(self._h, _ptr(out), _stream(stream)), "mbl_basis_states")
        return out.to(torch.int64) & 0xFFFFFFFF

    def rank(self, states, stream=None):
        import torch
        s32 = (states.to(torch.int64) & 0xFFFFFFFF).to(torch.int32).contiguous()
        out = torch.empty(s32.numel(), dtype=torch.int64, device="cuda")
        _check(lib.mbl_basis_rank(self._h, _ptr(s32), s32.numel(), _ptr(out), _stream(stream)),
               "mbl_basis_rank")
        return out


class Workspace:
    def __init__(self, basis: Basis, mmax: int = 0, precision: str = "fp64"):
        h = C.c_void_p()
        _check(lib.mbl_workspace_create(basis.handle, int(mmax), PRECISION[precision],
                                        C.byref(h)), "mbl_workspace_create", warn_ok=False)
        self._h = h
        self.basis = basis
        self.mmax = int(mmax)
        b = C.c_int64()
        _check(lib.mbl_workspace_bytes(h, C.byref(b)), "mbl_workspace_bytes")
        self.bytes = int(b.value)

    @property
    def handle(self):
        return self._h

    def __del__(self):
        if getattr(self, "_h", None) and lib is not None:
            try:
                lib.mbl_workspace_free(self._h)
            except Exception:   # interpreter shutdown
                pass
            self._h = None


def apply_H(basis: Basis, h, sigma: float, x, y=None, stream=None):
    """y = (H - sigma I) x for FP64 or FP32 x."""
    import torch
    if x.dtype not in (torch.float64, torch.float32):
        raise ValueError("x must be float64 or float32")
    _need_cuda(x, x.dtype, basis.n, "x")
    if y is None:
        y = torch.empty_like(x)
    _need_cuda(y, x.dtype, basis.n, "y")
    ha, hp = _f64(h)
    fn = lib.mbl_apply_H if x.dtype == torch.float64 else lib.mbl_apply_H_f32
    _check(fn(basis.handle, hp, float(sigma), _ptr(x), _ptr(y), _stream(stream)), "mbl_apply_H")
    return y


def precond_apply(basis: Basis, h, sigma: float, z, q=None, kind: str = "row", stream=None):
    import torch
    _need_cuda(z, torch.float64, basis.n, "z")
    if q is None:
        q = torch.empty_like(z)
    ha, hp = _f64(h)
    _check(lib.mbl_precond_apply(basis.handle, hp, float(sigma), PRECOND[kind], _ptr(z), _ptr(q),
                                 _stream(stream)), "mbl_precond_apply")
    return q


@dataclass
class SolveInfo:
    status: int
    iters: int
    restarts: int
    phi: float
    true_res: float


def minres_solve(basis: Basis, h, sigma: float, b, x=None, tol: float = 1e-12,
                 kmax: int = 10_000_000, precision: str = "fp64", precond: str = "row",
                 ws: Workspace | None = None, stream=None):
    """Preconditioned MINRES for (H - sigma) x = b (Alg. 2). Returns (x, info)."""
    import torch
    _need_cuda(b, torch.float64, basis.n, "b")
    if x is None:
        x = torch.zeros_like(b)
    _need_cuda(x, torch.float64, basis.n, "x")
    ws = ws or Workspace(basis, 0, precision)
    ha, hp = _f64(h)
    info = MinresInfo()
    st = lib.mbl_minres_solve(basis.handle, hp, float(sigma), _ptr(b), _ptr(x), float(tol),
                              int(kmax), PRECISION[precision], PRECOND[precond], ws.handle,
                              C.byref(info), _stream(stream))
    _check(st, "mbl_minres_solve")
    return x, SolveInfo(st, info.iters, info.restarts, info.phi, info.true_res)


@dataclass
class EigResult:
    status: int
    evals: np.ndarray
    evecs: object          # torch (n, nev) view of column-major storage
    resid: np.ndarray
    steps: int
    nconv: int
    minres_iters: int
    max_rel_resid: float
    seconds: float


def si_lanczos(basis: Basis, h, sigma: float, nev: int, mmax: int | None = None,
               minres_tol: float = 1e-12, minres_kmax: int = 10_000_000,
               eig_tol: float = 1e-10, gap_tol: float = 1e-5, escale: float = 0.0,
               v0=None, seed: int = 0, precision: str = "fp64", precond: str = "row",
               ws: Workspace | None = None, stream=None) -> EigResult:
    """The nev eigenpairs nearest sigma by shift-invert Lanczos (Alg. 1)."""
    import torch
    if mmax is None:
        mmax = min(basis.n, 3 * nev + 40)
    ws = ws if ws is not None else Workspace(basis, mmax, precision)
    if v0 is not None:
        _need_cuda(v0, torch.float64, basis.n, "v0")
    store = torch.empty((nev, basis.n), dtype=torch.float64, device="cuda")
    evals = np.zeros(nev)
    resid = np.zeros(nev)
    info = SiInfo()
    ha, hp = _f64(h)
    st = lib.mbl_si_lanczos(basis.handle, hp, float(sigma), int(nev), int(mmax), float(minres_tol),
                            int(minres_kmax), float(eig_tol), float(gap_tol), float(escale),
                            _ptr(v0) if v0 is not None else None, int(seed) & (2**64 - 1),
                            PRECISION[precision], PRECOND[precond], ws.handle,
                            evals.ctypes.data_as(_dp), _ptr(store), basis.n,
                            resid.ctypes.data_as(_dp), C.byref(info), _stream(stream))
    _check(st, "mbl_si_lanczos")
    return EigResult(st, evals, store.t(), resid, info.steps, info.nconv, info.minres_iters,
                     info.max_rel_resid, info.seconds)


def twist_expect(basis: Basis, psi, stream=None) -> np.ndarray:
    """z_t = <psi_t|U_twist|psi_t> for the columns of psi (n,) or (n, nvec)."""
    import torch
    if psi.dim() == 1:
        psi = psi[:, None]
    # column-major storage with leading dimension n
    store = psi.t().contiguous() if not psi.t().is_contiguous() else psi.t()
    _need_cuda(store, torch.float64, None, "psi")
    nvec = store.shape[0]
    z = np.zeros(2 * nvec)
    _check(lib.mbl_twist_expect(basis.handle, _ptr(store), basis.n, nvec, z.ctypes.data_as(_dp),
                                _stream(stream)), "mbl_twist_expect")
    return z[0::2] + 1j * z[1::2]


def entanglement_entropy(basis: Basis, psi, la: int | None = None, stream=None) -> np.ndarray:
    """S_t = -Tr rho_A ln rho_A, A = sites 1..la (default L/2), for the
    columns of psi (n,) or (n, nvec) (Sec. IV)."""
    import torch
    if psi.dim() == 1:
        psi = psi[:, None]
    store = psi.t().contiguous() if not psi.t().is_contiguous() else psi.t()
    _need_cuda(store, torch.float64, None, "psi")
    nvec = store.shape[0]
    S = np.zeros(nvec)
    la = basis.L // 2 if la is None else int(la)
    _check(lib.mbl_entanglement_entropy(basis.handle, _ptr(store), basis.n, nvec, la,
                                        S.ctypes.data_as(_dp), _stream(stream)),
           "mbl_entanglement_entropy")
    return S


def entanglement_entropy_batched(basis: Basis, U, la: int | None = None, stream=None):
    """S[r, t] for the (nev, n, R) interleaved eigenvector blocks of
    si_lanczos_batched (A = sites 1..la, default L/2)."""
    import torch
    if U.dim() == 2:
        U = U[None]
    _need_cuda(U, torch.float64, None, "U")
    if not U.is_contiguous():
        raise ValueError("U must be contiguous (nev, n, R)")
    nvec, n, R = U.shape
    if n != basis.n:
        raise ValueError("U must be (nev, n, R) with n the basis dimension")
    S = np.zeros(R * nvec)
    la = basis.L // 2 if la is None else int(la)
    _check(lib.mbl_entanglement_entropy_interleaved(basis.handle, _ptr(U), R, nvec, la,
                                                    S.ctypes.data_as(_dp), _stream(stream)),
           "mbl_entanglement_entropy_interleaved")
    return S.reshape(R, nvec)


def symmetric_eigenvalues(A) -> np.ndarray:
    """Ascending eigenvalues of a symmetric matrix, by the host routine the
    entanglement entropy uses for its Schmidt blocks."""
    A, Ap = _f64(A)
    m = A.shape[0]
    if A.ndim != 2 or A.shape != (m, m):
        raise ValueError("A must be square")
    w = np.zeros(m)
    _check(lib.mbl_symmetric_eigenvalues(m, Ap, w.ctypes.data_as(_dp)), "mbl_symmetric_eigenvalues")
    return w


def spacing_ratio(evals):
    """(mean r, r_k) of the level-spacing ratios of the sorted eigenvalues (Sec. IV)."""
    E, Ep = _f64(np.ravel(evals))
    r = np.zeros(max(len(E) - 2, 1))
    mean = C.c_double()
    _check(lib.mbl_spacing_ratio(len(E), Ep, r.ctypes.data_as(_dp), C.byref(mean)),
           "mbl_spacing_ratio")
    return mean.value, r[:len(E) - 2]


def eig_residual(basis: Basis, h, E, psi, stream=None) -> np.ndarray:
    import torch
    if psi.dim() == 1:
        psi = psi[:, None]
    store = psi.t().contiguous() if not psi.t().is_contiguous() else psi.t()
    _need_cuda(store, torch.float64, None, "psi")
    nvec = store.shape[0]
    Ea, Ep = _f64(np.atleast_1d(E))
    out = np.zeros(nvec)
    ha, hp = _f64(h)
    _check(lib.mbl_eig_residual(basis.handle, hp, Ep, _ptr(store), basis.n, nvec,
                                out.ctypes.data_as(_dp), _stream(stream)), "mbl_eig_residual")
    return out


def sigma_midpoint(basis: Basis, h, rel_tol: float = 1e-12, mmax: int = 0, stream=None):
    """(E_min, E_max, sigma = (E_min + E_max)/2)."""
    ha, hp = _f64(h)
    lo, hi, sg = C.c_double(), C.c_double(), C.c_double()
    _check(lib.mbl_sigma_midpoint(basis.handle, hp, float(rel_tol), int(mmax), C.byref(lo),
                                  C.byref(hi), C.byref(sg), _stream(stream)), "mbl_sigma_midpoint")
    return lo.value, hi.value, sg.value


def dot(x, y, stream=None) -> float:
    import torch
    _need_cuda(x, torch.float64, None, "x")
    _need_cuda(y, torch.float64, x.numel(), "y")
    out = C.c_double()
    _check(lib.mbl_dot(x.numel(), _ptr(x), _ptr(y), C.byref(out), _stream(stream)), "mbl_dot")
    return out.value


def tridiag_eig(alpha, beta):
    """Host-only eigen-decomposition of the Lanczos tridiagonal T_k."""
    a, ap = _f64(alpha)
    k = a.shape[0]
    b, bp = _f64(beta if k > 1 else np.zeros(1))
    w = np.zeros(k)
    V = np.zeros(k * k)
    _check(lib.mbl_tridiag_eig(k, ap, bp, w.ctypes.data_as(_dp), V.ctypes.data_as(_dp)),
           "mbl_tridiag_eig", warn_ok=False)
    return w, V.reshape(k, k).T


# ---------------------------------------------------------------- batched form
_sig("mbl_batch_create", _i32, [_vp, C.c_int, C.c_int, C.c_int, C.POINTER(_vp)])
_sig("mbl_batch_free", None, [_vp])
_sig("mbl_batch_bytes", _i32, [_vp, C.POINTER(C.c_int64)])
_sig("mbl_batch_set_schedule", _i32, [_vp, C.c_int, C.c_int, C.c_int])
_sig("mbl_apply_H_batched", _i32, [_vp, _vp, _dp, _dp, _vp, _vp, _vp])
_sig("mbl_apply_H_batched_f32", _i32, [_vp, _vp, _dp, _dp, _vp, _vp, _vp])
_sig("mbl_minres_solve_batched", _i32, [_vp, _vp, _dp, _dp, _vp, _vp, _d, _i64, C.c_int, C.c_int,
                                        C.POINTER(C.c_int64), _dp, _vp])
_sig("mbl_si_lanczos_batched", _i32, [_vp, _vp, _dp, _dp, C.c_int, C.c_int, _d, _i64, _d, _d, _dp,
                                      _vp, _u64, C.c_int, C.c_int, _dp, _vp, _dp,
                                      C.POINTER(SiInfo), _vp])
_sig("mbl_twist_expect_batched", _i32, [_vp, _vp, _vp, C.c_int, _dp, _vp])


class Batch:
    """Workspace for R realizations of one L solved together. Batched
    vectors are (n, R) row-major tensors: element (i, r) at i * R + r."""

    def __init__(self, basis: Basis, R: int, mmax: int = 0, nevmax: int = 0):
        h = C.c_void_p()
        _check(lib.mbl_batch_create(basis.handle, int(R), int(mmax), int(nevmax), C.byref(h)),
               "mbl_batch_create", warn_ok=False)
        self._h = h
        self.basis = basis
        self.R = int(R)
        self.mmax = int(mmax)
        self.nevmax = int(nevmax)
        b = C.c_int64()
        _check(lib.mbl_batch_bytes(h, C.byref(b)), "mbl_batch_bytes")
        self.bytes = int(b.value)

    @property
    def handle(self):
        return self._h

    def set_schedule(self, grid: int = 0, graph_iters: int = 0, dx_group: int = 0):
        """Launch schedule of the batched kernels (mbl_batch_set_schedule);
        0 keeps the library's default for that knob."""
        _check(lib.mbl_batch_set_schedule(self._h, int(grid), int(graph_iters), int(dx_group)),
               "mbl_batch_set_schedule", warn_ok=False)
        self.schedule = (int(grid), int(graph_iters), int(dx_group))

    def __del__(self):
        if getattr(self, "_h", None) and lib is not None:
            try:
                lib.mbl_batch_free(self._h)
            except Exception:   # interpreter shutdown
                pass
            self._h = None


def _fields_matrix(h_list, R, L):
    H = np.ascontiguousarray(np.asarray(h_list, dtype=np.float64).reshape(R, L))
    return H, H.ctypes.data_as(_dp)


def apply_H_batched(basis: Basis, batch: Batch, fields, sigmas, x, y=None, stream=None):
    """y[:, r] = (H_r - sigma_r) x[:, r] for the (n, R) interleaved x."""
    import torch
    if x.dtype not in (torch.float64, torch.float32):
        raise ValueError("x must be float64 or float32")
    _need_cuda(x, x.dtype, basis.n * batch.R, "x")
    if y is None:
        y = torch.empty_like(x)
    _need_cuda(y, x.dtype, basis.n * batch.R, "y")
    H, hp = _fields_matrix(fields, batch.R, basis.L)
    sg, sp = _f64(sigmas)
    fn = lib.mbl_apply_H_batched if x.dtype == torch.float64 else lib.mbl_apply_H_batched_f32
    _check(fn(basis.handle, batch.handle, hp, sp, _ptr(x), _ptr(y), _stream(stream)),
           "mbl_apply_H_batched")
    return y


def minres_solve_batched(basis: Basis, batch: Batch, fields, sigmas, b, x=None, tol=1e-12,
                         kmax=10_000_000, precision="fp64", precond="row", stream=None):
    import torch
    _need_cuda(b, torch.float64, basis.n * batch.R, "b")
    if x is None:
        x = torch.zeros_like(b)
    H, hp = _fields_matrix(fields, batch.R, basis.L)
    sg, sp = _f64(sigmas)
    its = (C.c_int64 * batch.R)()
    phi = np.zeros(batch.R)
    st = lib.mbl_minres_solve_batched(basis.handle, batch.handle, hp, sp, _ptr(b), _ptr(x),
                                      float(tol), int(kmax), PRECISION[precision], PRECOND[precond],
                                      its, phi.ctypes.data_as(_dp), _stream(stream))
    _check(st, "mbl_minres_solve_batched")
    return x, np.array(list(its), dtype=np.int64), phi, st


@dataclass
class BatchEigResult:
    status: int
    evals: np.ndarray        # (R, nev)
    evecs: object            # torch (nev, n, R)
    resid: np.ndarray        # (R, nev)
    steps: np.ndarray        # (R,)
    nconv: np.ndarray        # (R,)
    minres_iters: int        # whole batch: the sum of per_realization_iters
    max_rel_resid: np.ndarray
    seconds: float
    per_realization_iters: np.ndarray   # (R,) each realization's own MINRES iterations


def si_lanczos_batched(basis: Basis, batch: Batch, fields, sigmas, nev: int, mmax: int | None = None,
                       minres_tol=1e-12, minres_kmax=10_000_000, eig_tol=1e-10, gap_tol=1e-5,
                       escale=None, v0=None, seed=0, precision="fp64", precond="row",
                       stream=None) -> BatchEigResult:
    import torch
    R, n = batch.R, basis.n
    if mmax is None:
        mmax = min(batch.mmax, 3 * nev + 40)
    H, hp = _fields_matrix(fields, R, basis.L)
    sg, sp = _f64(sigmas)
    es = None
    if escale is not None:
        esa, es = _f64(escale)
    if v0 is not None:
        _need_cuda(v0, torch.float64, n * R, "v0")
    U = torch.empty((nev, n, R), dtype=torch.float64, device="cuda")
    evals = np.zeros(R * nev)
    resid = np.zeros(R * nev)
    info = (SiInfo * R)()
    st = lib.mbl_si_lanczos_batched(basis.handle, batch.handle, hp, sp, int(nev), int(mmax),
                                    float(minres_tol), int(minres_kmax), float(eig_tol),
                                    float(gap_tol), es, _ptr(v0) if v0 is not None else None,
                                    int(seed) & (2**64 - 1), PRECISION[precision],
                                    PRECOND[precond], evals.ctypes.data_as(_dp), _ptr(U),
                                    resid.ctypes.data_as(_dp), info, _stream(stream))
    _check(st, "mbl_si_lanczos_batched")
    return BatchEigResult(st, evals.reshape(R, nev), U, resid.reshape(R, nev),
                          np.array([i.steps for i in info]), np.array([i.nconv for i in info]),
                          int(sum(i.minres_iters for i in info)),
                          np.array([i.max_rel_resid for i in info]), float(info[0].seconds),
                          np.array([i.minres_iters for i in info], dtype=np.int64))


def twist_expect_batched(basis: Basis, batch: Batch, U, stream=None) -> np.ndarray:
    """z[r, t] for the (nev, n, R) interleaved eigenvector blocks."""
    import torch
    if U.dim() == 2:
        U = U[None]
    _need_cuda(U, torch.float64, None, "U")
    nvec = U.shape[0]
    z = np.zeros(batch.R * nvec * 2)
    _check(lib.mbl_twist_expect_batched(basis.handle, batch.handle, _ptr(U), nvec,
                                        z.ctypes.data_as(_dp), _stream(stream)),
           "mbl_twist_expect_batched")
    z = z.reshape(batch.R, nvec, 2)
    return z[..., 0] + 1j * z[..., 1]


# ---------------------------------------------------------------- derivatives
_sig("mbl_eig_grad", _i32, [_vp, _dp, _d, _vp, _d, _i64, C.c_int, _vp, _dp, _dp, _dp,
                            C.POINTER(MinresInfo), _vp])


class Problem(C.Structure):
    """mbl_problem of include/mbl.h."""
    _fields_ = [("L", C.c_int32), ("nev", C.c_int32), ("h_host", _dp), ("sigma", C.c_double),
                ("escale", C.c_double), ("evecs_dev", _vp), ("evals_host", _dp),
                ("resid_host", _dp), ("z_host", _dp), ("sigma_out", C.c_double),
                ("info", SiInfo), ("status", C.c_int32)]


_sig("mbl_si_lanczos_problems", _i32, [C.POINTER(Problem), C.c_int, C.c_int, _d, _i64, _d, _d,
                                       _u64, C.c_int, _vp])


@dataclass
class ProblemResult:
    L: int
    status: int
    evals: np.ndarray
    evecs: object          # torch (n, nev) view of column-major storage
    resid: np.ndarray
    z: np.ndarray
    sigma: float
    steps: int
    nconv: int
    minres_iters: int
    max_rel_resid: float
    seconds: float


def si_lanczos_problems(problems, mmax: int = 0, minres_tol: float = 1e-12,
                        minres_kmax: int = 10_000_000, eig_tol: float = 1e-10,
                        gap_tol: float = 1e-5, seed: int = 0, precond: str = "row", stream=None):
    """Eigenpairs nearest sigma of many realizations of uneven L in one call
    (mbl_si_lanczos_problems). problems: sequence of dicts with keys L, h, nev
    and optionally sigma (default: the spectral midpoint, computed) and
    escale. Returns (status, [ProblemResult])."""
    import torch
    keep, arr = [], (Problem * len(problems))()
    out = []
    for i, p in enumerate(problems):
        L, nev = int(p["L"]), int(p["nev"])
        n = math.comb(L, L // 2)
        ha, hp = _f64(p["h"])
        if ha.shape[0] != L:
            raise ValueError("h must hold L fields")
        store = torch.empty((nev, n), dtype=torch.float64, device="cuda")
        ev, rs, zz = np.zeros(nev), np.zeros(nev), np.zeros(2 * nev)
        keep += [ha, store, ev, rs, zz]
        a = arr[i]
        a.L, a.nev, a.h_host = L, nev, hp
        a.sigma = float(p.get("sigma", float("nan")))
        a.escale = float(p.get("escale", 0.0))
        a.evecs_dev = store.data_ptr()
        a.evals_host, a.resid_host, a.z_host = (ev.ctypes.data_as(_dp), rs.ctypes.data_as(_dp),
                                                zz.ctypes.data_as(_dp))
        out.append((store, ev, rs, zz))
    st = lib.mbl_si_lanczos_problems(arr, len(problems), int(mmax), float(minres_tol),
                                     int(minres_kmax), float(eig_tol), float(gap_tol),
                                     int(seed) & (2**64 - 1), PRECOND[precond], _stream(stream))
    _check(st, "mbl_si_lanczos_problems")
    res = []
    for i, (store, ev, rs, zz) in enumerate(out):
        a = arr[i]
        res.append(ProblemResult(int(a.L), int(a.status), ev, store.t(), rs, zz[0::2] + 1j * zz[1::2],
                                 float(a.sigma_out), int(a.info.steps), int(a.info.nconv),
                                 int(a.info.minres_iters), float(a.info.max_rel_resid),
                                 float(a.info.seconds)))
    return st, res


def eig_grad(basis: Basis, h, E: float, psi, tol: float = 1e-10, kmax: int = 10_000_000,
             precond: str = "row", ws: Workspace | None = None, stream=None):
    """(dE/dh, d|z|^2/dh, z, info) for the eigenpair (E, psi), psi an (n,) FP64 tensor."""
    import torch
    _need_cuda(psi, torch.float64, basis.n, "psi")
    ws = ws or Workspace(basis, 0)
    L = basis.L
    dE = np.zeros(L)
    dz2 = np.zeros(L)
    z = np.zeros(2)
    info = MinresInfo()
    ha, hp = _f64(h)
    st = lib.mbl_eig_grad(basis.handle, hp, float(E), _ptr(psi), float(tol), int(kmax),
                          PRECOND[precond], ws.handle, dE.ctypes.data_as(_dp),
                          dz2.ctypes.data_as(_dp), z.ctypes.data_as(_dp), C.byref(info),
                          _stream(stream))
    _check(st, "mbl_eig_grad")
    return dE, dz2, complex(z[0], z[1]), SolveInfo(st, info.iters, info.restarts, info.phi,
                                                   info.true_res)


class EigPair:
    """Differentiable map h -> (E, |z|^2) of one eigenpair near sigma.

    ``EigPair(basis, sigma, nev, which)(h)`` runs shift-invert Lanczos for the
    nev pairs nearest sigma and returns the eigenvalue and |z|^2 of pair
    ``which`` (ascending order) as torch scalars; backward() obtains dE/dh
    (Hellmann-Feynman) and d|z|^2/dh (one adjoint MINRES solve) from the
    library. ``h`` is a float64 CPU or GPU tensor of length L."""

    def __init__(self, basis: Basis, sigma: float, nev: int = 1, which: int = 0,
                 grad_tol: float = 1e-10, **si_kw):
        self.basis, self.sigma, self.nev, self.which = basis, sigma, nev, which
        self.grad_tol, self.si_kw = grad_tol, si_kw

    def __call__(self, h):
        return _EigPairFn.apply(h, self)


def _make_fn():
    import torch

    class _Fn(torch.autograd.Function):
        @staticmethod
        def forward(ctx, h, spec):
            hh = h.detach().cpu().numpy().astype(np.float64)
            res = si_lanczos(spec.basis, hh, spec.sigma, spec.nev, **spec.si_kw)
            psi = res.evecs[:, spec.which].contiguous()
            E = float(res.evals[spec.which])
            z = twist_expect(spec.basis, psi)[0]
            ctx.spec, ctx.E, ctx.hh = spec, E, hh
            ctx.psi = psi
            ctx.h_device = h.device
            return (torch.tensor(E, dtype=torch.float64, device=h.device),
                    torch.tensor(abs(z) ** 2, dtype=torch.float64, device=h.device))

        @staticmethod
        def backward(ctx, gE, gz2):
            dE, dz2, _, _ = eig_grad(ctx.spec.basis, ctx.hh, ctx.E, ctx.psi, tol=ctx.spec.grad_tol)
            gh = (gE.detach().cpu().double() * torch.from_numpy(dE)
                  + gz2.detach().cpu().double() * torch.from_numpy(dz2))
            return gh.to(ctx.h_device), None

    return _Fn


_EigPairFn = _make_fn()
