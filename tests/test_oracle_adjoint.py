"""Pins for the oracle's eigenpair derivatives."""
import numpy as np
import pytest

from oracle import adjoint, model, twist
from workloads import disorder_fields


@pytest.mark.parametrize("L,seed,which", [(8, 0, 30), (10, 1, 120)])
def test_hellmann_feynman_and_perturbation_sum_vs_finite_differences(L, seed, which):
    h = disorder_fields(L, 3.0, seed)
    E, psi, dpsi = adjoint.eigvec_derivatives(L, h, which)
    dE_hf = adjoint.hellmann_feynman(L, psi)
    dz2 = adjoint.dz2_dh(L, psi, dpsi)
    dE_fd, dz2_fd = adjoint.finite_difference(L, h, E, step=1e-5)
    # central differences carry an O(step^2 / gap^2) truncation error
    assert np.abs(dE_hf - dE_fd).max() < 1e-6
    assert np.abs(dz2 - dz2_fd).max() < 1e-5 * max(1.0, np.abs(dz2).max())
    # a uniform shift of all fields changes nothing in S^z_tot = 0
    assert abs(dE_hf.sum()) < 1e-12
    assert abs(dz2.sum()) < 1e-9
    # the derivative is orthogonal to psi (normalisation is kept)
    assert np.abs(psi @ dpsi).max() < 1e-12
