"""Pins of the oracle's eigenstate observables (Sec. IV, entanglement and
level spacing) against closed forms that do not go through its SVD."""
import math

import numpy as np
import pytest

from oracle import model, observables


def _sector_vector(L, amplitudes):
    """Sector vector from {state integer: amplitude}."""
    states = model.sector_states(L)
    v = np.zeros(states.shape[0])
    for s, a in amplitudes.items():
        i = int(np.searchsorted(states, s))
        assert states[i] == s
        v[i] += a
    return v


def _singlets(L, pairs):
    """Product of singlets (|up down> - |down up>)/sqrt 2 on the given site
    pairs (1-based; the first site of a pair up gives +)."""
    amps = {}
    for choice in range(1 << len(pairs)):
        s, a = 0, 1.0
        for t, (i, j) in enumerate(pairs):
            if (choice >> t) & 1:
                s |= 1 << (j - 1)
                a *= -1 / math.sqrt(2)
            else:
                s |= 1 << (i - 1)
                a *= 1 / math.sqrt(2)
        amps[s] = a
    return _sector_vector(L, amps)


@pytest.mark.parametrize("L", [4, 6, 8, 10])
def test_basis_state_has_zero_entropy(L):
    states = model.sector_states(L)
    for idx in (0, len(states) // 3, len(states) - 1):
        v = np.zeros(len(states))
        v[idx] = 1.0
        for la in range(1, L):
            assert abs(observables.entanglement_entropy(L, v, la)) < 1e-14


@pytest.mark.parametrize("L", [4, 6, 8, 10])
def test_mirror_singlets_give_la_ln2(L):
    """Singlets on (j, L+1-j): for la <= L/2 every site of A is paired with
    a site of B, so S = la ln 2 (and S(la) = S(L - la))."""
    v = _singlets(L, [(j, L + 1 - j) for j in range(1, L // 2 + 1)])
    assert abs(np.linalg.norm(v) - 1) < 1e-14
    for la in range(1, L):
        want = min(la, L - la) * math.log(2)
        assert abs(observables.entanglement_entropy(L, v, la) - want) < 1e-12


def test_singlets_count_only_bonds_across_the_cut():
    """Pairs (1,2), (3,5), (4,6) at L = 6: the cut after site la crosses
    0, 1, 2, 1 singlets for la = 2, 3, 4, 5 (A = sites 1..la; the far end
    of the chain would give 2, 1, 0, ... instead)."""
    v = _singlets(6, [(1, 2), (3, 5), (4, 6)])
    for la, crossing in ((1, 1), (2, 0), (3, 1), (4, 2), (5, 1)):
        assert abs(observables.entanglement_entropy(6, v, la) - crossing * math.log(2)) < 1e-12


def test_two_state_superpositions():
    """cos t |a1 b1> + sin t |a2 b2>: Schmidt weights cos^2, sin^2 when both
    halves differ; a product state (S = 0) when only A differs."""
    L, la, t = 8, 4, 0.37
    a1, a2 = 0b0011, 0b0101          # sites 1..4, two up spins each
    b1, b2 = 0b1100, 0b0110          # sites 5..8
    c, s = math.cos(t), math.sin(t)
    v = _sector_vector(L, {a1 | (b1 << la): c, a2 | (b2 << la): s})
    want = -(c * c * math.log(c * c) + s * s * math.log(s * s))
    assert abs(observables.entanglement_entropy(L, v, la) - want) < 1e-13
    v = _sector_vector(L, {a1 | (b1 << la): c, a2 | (b1 << la): s})
    assert abs(observables.entanglement_entropy(L, v, la)) < 1e-13


@pytest.mark.parametrize("L,la", [(6, 3), (8, 3), (10, 5), (12, 4)])
def test_uniform_superposition_hypergeometric(L, la):
    """Equal amplitudes on every sector state: each magnetisation block of
    the coefficient matrix is rank one, with weight C(la, k) C(L-la, L/2-k)
    / C(L, L/2), so S is the entropy of that distribution."""
    n = math.comb(L, L // 2)
    v = np.full(n, 1.0)     # unnormalised on purpose
    p = [math.comb(la, k) * math.comb(L - la, L // 2 - k) / n for k in range(0, la + 1)]
    want = -sum(q * math.log(q) for q in p if q > 0)
    assert abs(observables.entanglement_entropy(L, v, la) - want) < 1e-12


def test_random_vector_reflection_and_scale():
    """S(A) = S(B): the chain reflected (site j -> L + 1 - j) and scaled has
    at cut L - la the entropy of the original at cut la."""
    rng = np.random.default_rng(5)
    L = 10
    states = model.sector_states(L)
    v = rng.standard_normal(states.shape[0])
    rev = np.array([int(format(int(s), f"0{L}b")[::-1], 2) for s in states])
    vr = np.zeros_like(v)
    vr[np.searchsorted(states, rev)] = v
    for la in range(1, L):
        s1 = observables.entanglement_entropy(L, v, la)
        s2 = observables.entanglement_entropy(L, 3.7 * vr, L - la)
        assert abs(s1 - s2) < 1e-12
    # S never exceeds the log of the smaller side's sector-resolved dimension
    assert observables.entanglement_entropy(L, v) <= (L // 2) * math.log(2)


def test_spacing_ratio_small_cases():
    assert np.allclose(observables.spacing_ratios(np.arange(7.0)), 1.0)
    assert np.allclose(observables.spacing_ratios([0.0, 1.0, 3.0, 3.5]), [0.5, 0.25])
    assert np.allclose(observables.spacing_ratios([3.5, 0.0, 3.0, 1.0]), [0.5, 0.25])
    r = observables.spacing_ratios([0.0, 1.0, 1.0, 1.0, 2.0])
    assert np.isnan(r[1]) and r[0] == 0.0 and r[2] == 0.0
    assert observables.mean_spacing_ratio([0.0, 1.0, 1.0, 1.0, 2.0]) == 0.0


def test_spacing_ratio_poisson_value():
    """Independent levels (exponential spacings): <r> = 2 ln 2 - 1."""
    rng = np.random.default_rng(11)
    E = rng.uniform(0, 1, 400_000)
    assert abs(observables.mean_spacing_ratio(E) - (2 * math.log(2) - 1)) < 2e-3


def test_spacing_ratio_goe_value():
    """Central levels of GOE matrices: <r> = 0.5307 (large-N value)."""
    rng = np.random.default_rng(12)
    rs = []
    for _ in range(30):
        A = rng.standard_normal((400, 400))
        w = np.linalg.eigvalsh(A + A.T)
        rs.extend(observables.spacing_ratios(w[100:300]))
    assert abs(np.mean(rs) - 0.5307) < 0.01
