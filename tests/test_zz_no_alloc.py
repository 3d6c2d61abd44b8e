"""The allocation-free twist overlap against mbl_twist_expect, through the C
ABI: two calls in a row, the second with a smaller input (another basis, fewer
vectors), each bit for bit equal to the allocating entry point; the size
limit (nvec <= 32) is rejected with MBL_ERR_ARG and a message."""
import ctypes as C
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _noalloc(mbl, b, store, nvec):
    z = np.full(2 * nvec, np.nan)
    st = mbl.lib.mbl_twist_expect_noalloc(b.handle, C.c_void_p(store.data_ptr()), b.n, nvec,
                                          z.ctypes.data_as(C.POINTER(C.c_double)), None)
    return st, z[0::2] + 1j * z[1::2]


def _case(mbl, torch, L, nvec, seed):
    b = mbl.Basis(L)
    g = torch.Generator(device="cuda").manual_seed(seed)
    store = torch.randn((nvec, b.n), dtype=torch.float64, device="cuda", generator=g)
    store /= store.norm(dim=1, keepdim=True)
    say(f"noalloc twist L={L} nvec={nvec}")
    torch.cuda.synchronize()
    st, z = _noalloc(mbl, b, store, nvec)
    assert st == mbl.OK, mbl.lib.mbl_last_error().decode()
    zref = mbl.twist_expect(b, store.t())
    assert np.array_equal(z, zref), np.abs(z - zref).max()
    return b, store


def test_twist_noalloc_matches_allocating_call(gpu):
    import torch
    mbl = gpu
    _case(mbl, torch, 18, 32, 1)       # the largest call the static scratch holds
    b, store = _case(mbl, torch, 12, 3, 2)   # then a smaller one: stale partials must not leak
    # beyond the static scratch: rejected before any launch
    big = torch.zeros((33, b.n), dtype=torch.float64, device="cuda")
    st, z = _noalloc(mbl, b, big, 33)
    assert st == mbl.ERR_ARG and "32" in mbl.lib.mbl_last_error().decode()
    assert np.all(np.isnan(z))
    st, _ = _noalloc(mbl, b, store, 0)
    assert st == mbl.ERR_ARG
