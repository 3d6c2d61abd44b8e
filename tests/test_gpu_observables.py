"""Entanglement entropy (Sec. IV) on the device against the oracle's
Schmidt decomposition, and the level-spacing ratio through the library."""
import math
import sys

import numpy as np
import pytest

from oracle import model, observables
from workloads import disorder_fields, gaussian_vector

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


def dev(torch, a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda")


@pytest.mark.parametrize("L", [4, 6, 8, 10])
def test_entropy_every_cut_small(gpu, torch, L):
    """Random vectors (three at once), every cut 1..L-1, against the oracle."""
    say(f"entropy L={L} every cut")
    b = gpu.Basis(L)
    V = np.stack([gaussian_vector(b.n, 60 + t) for t in range(3)], axis=1)
    Vd = dev(torch, V)
    for la in range(1, L):
        S = gpu.entanglement_entropy(b, Vd, la)
        want = [observables.entanglement_entropy(L, V[:, t], la) for t in range(3)]
        assert np.abs(S - want).max() <= 1e-11, (la, S, want)


@pytest.mark.parametrize("L,las", [(12, (1, 4, 6, 9)), (14, (3, 7, 12)), (16, (5, 8)),
                                   (18, (9,)), (20, (7, 10))])
def test_entropy_larger_sizes(gpu, torch, L, las):
    say(f"entropy L={L} cuts {las}")
    b = gpu.Basis(L)
    v = gaussian_vector(b.n, 70 + L)
    vd = dev(torch, v)
    for la in las:
        S = gpu.entanglement_entropy(b, vd, la)[0]
        want = observables.entanglement_entropy(L, v, la)
        assert abs(S - want) <= 1e-10, (la, S, want)


@pytest.mark.parametrize("L", [8, 12, 16])
def test_entropy_closed_forms(gpu, torch, L):
    """Mirror singlets: S = min(la, L-la) ln 2; one basis state: S = 0; the
    uniform vector: the entropy of the hypergeometric block weights."""
    say(f"entropy closed forms L={L}")
    b = gpu.Basis(L)
    states = model.sector_states(L)
    pairs = [(j, L + 1 - j) for j in range(1, L // 2 + 1)]
    amps = {}
    for choice in range(1 << len(pairs)):
        s, a = 0, 1.0
        for t, (i, j) in enumerate(pairs):
            s |= 1 << ((j if (choice >> t) & 1 else i) - 1)
            a *= (-1 if (choice >> t) & 1 else 1) / math.sqrt(2)
        amps[s] = a
    sing = np.zeros(b.n)
    sing[np.searchsorted(states, list(amps))] = list(amps.values())
    one = np.zeros(b.n)
    one[b.n // 3] = 1.0
    uni = np.full(b.n, 2.5)
    V = dev(torch, np.stack([sing, one, uni], axis=1))
    for la in (1, L // 2 - 1, L // 2, L - 2):
        S = gpu.entanglement_entropy(b, V, la)
        p = [math.comb(la, k) * math.comb(L - la, L // 2 - k) / b.n for k in range(la + 1)
             if 0 <= L // 2 - k <= L - la]
        hyper = -sum(q * math.log(q) for q in p if q > 0)
        assert abs(S[0] - min(la, L - la) * math.log(2)) <= 1e-11
        assert abs(S[1]) <= 1e-12
        assert abs(S[2] - hyper) <= 1e-11


def test_entropy_of_eigenvectors_L14(gpu, torch):
    """Mid-spectrum eigenvectors from the library's shift-invert Lanczos:
    the entropies equal the oracle's on the same vectors, and at h = 0.5
    (ergodic side) their mean is within 0.5 of the random-state entropy of Sec. IV B."""
    L = 14
    say("entropy of SI-Lanczos eigenvectors L=14")
    b = gpu.Basis(L)
    h = disorder_fields(L, 0.5, 3)
    lo, hi, sigma = gpu.sigma_midpoint(b, h, 1e-10)
    res = gpu.si_lanczos(b, h, sigma, nev=6, escale=max(abs(lo), abs(hi)))
    U = res.evecs
    S = gpu.entanglement_entropy(b, U)
    Uh = U.detach().cpu().numpy()
    want = [observables.entanglement_entropy(L, Uh[:, t]) for t in range(Uh.shape[1])]
    assert np.abs(S - want).max() <= 1e-10
    assert abs(np.mean(S) - observables.rmt_entropy(L)) < 0.5


def test_entropy_errors(gpu, torch):
    b = gpu.Basis(8)
    v = dev(torch, np.zeros(b.n))
    with pytest.raises(gpu.MblError):
        gpu.entanglement_entropy(b, v, 4)          # zero vector
    w = dev(torch, gaussian_vector(b.n, 1))
    for la in (0, 8):
        with pytest.raises(gpu.MblError):
            gpu.entanglement_entropy(b, w, la)


def test_entropy_nearly_product_states(gpu, torch):
    """Localised states: one or two basis states plus 1e-150 noise. Their
    Schmidt blocks have columns 1e-150 below the rest, which the host
    reduction must scale; S = 0 and S = ln 2 (the two states differ on both
    sides of the cut)."""
    L = 12
    say("entropy of nearly product states")
    b = gpu.Basis(L)
    states = model.sector_states(L)
    noise = 1e-150 * gaussian_vector(b.n, 5)
    v1 = noise.copy()
    v1[100] = 1.0
    a, c = 0b000111 | (0b111000 << 6), 0b111000 | (0b000111 << 6)
    v2 = noise.copy()
    v2[np.searchsorted(states, [a, c])] = 1.0 / math.sqrt(2)
    S = gpu.entanglement_entropy(b, dev(torch, np.stack([v1, v2], axis=1)))
    assert abs(S[0]) <= 1e-12 and abs(S[1] - math.log(2)) <= 1e-12


def test_entropy_leading_dimension_through_the_abi(gpu, torch):
    """Column-major storage with ld = n + 5 (padding poisoned with NaN),
    called through the C ABI: the padding is never read."""
    import ctypes as C
    L = 10
    b = gpu.Basis(L)
    ld, nvec = b.n + 5, 3
    V = np.full((nvec, ld), np.nan)
    for t in range(nvec):
        V[t, :b.n] = gaussian_vector(b.n, 90 + t)
    Vd = dev(torch, V)
    S = np.zeros(nvec)
    st = gpu.lib.mbl_entanglement_entropy(b.handle, C.c_void_p(Vd.data_ptr()), ld, nvec, 4,
                                          S.ctypes.data_as(C.POINTER(C.c_double)), None)
    assert st == 0
    want = [observables.entanglement_entropy(L, V[t, :b.n], 4) for t in range(nvec)]
    assert np.abs(S - want).max() <= 1e-11


def test_entropy_of_batched_eigenvectors(gpu, torch):
    """Interleaved eigenvector blocks of the batched SI-Lanczos: the batched
    entry point equals the single one on each de-interleaved vector bit for
    bit, and the oracle's SVD to the parity bar."""
    L, R, nev = 12, 4, 4
    say("entropy of batched eigenvectors L=12 R=4")
    b = gpu.Basis(L)
    bt = gpu.Batch(b, R, mmax=60, nevmax=nev)
    fields = [disorder_fields(L, 2.0 + 0.5 * r, 30 + r) for r in range(R)]
    sig, esc = [], []
    for f in fields:
        lo, hi, sg = gpu.sigma_midpoint(b, f, 1e-12)
        sig.append(sg)
        esc.append(max(abs(lo), abs(hi)))
    res = gpu.si_lanczos_batched(b, bt, fields, sig, nev, escale=esc)
    for la in (L // 2, 3):
        Sb = gpu.entanglement_entropy_batched(b, res.evecs, la)
        assert Sb.shape == (R, nev)
        for r in range(R):
            U = res.evecs[:, :, r].t().contiguous()
            Ss = gpu.entanglement_entropy(b, U, la)
            assert np.array_equal(Sb[r], Ss)
            Uh = U.cpu().numpy()
            want = [observables.entanglement_entropy(L, Uh[:, t], la) for t in range(nev)]
            assert np.abs(Sb[r] - want).max() <= 1e-10
