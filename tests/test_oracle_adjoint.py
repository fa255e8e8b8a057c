"""Pins of the oracle's implicit-function adjoint (vector-Jacobian product of
the projection with respect to u_hat)."""
import numpy as np
import pytest

from oracle.families import BurgersLF, FisherKPP, MassIC
from oracle.kkt import adjoint_sample, project_sample
from test_oracle_pins import _all_tiny, fd_jac, probe_affine


def test_linear_adjoint_is_the_null_space_projector():
    rng = np.random.default_rng(4)
    for fam in (MassIC(6, 4, rng.standard_normal(6)),
                FisherKPP(5, 4, rng.uniform(0.2, 0.8, 5), rho=0.0, dt=0.1),
                BurgersLF(5, 4, 0.01, 0.2, 0.01, 1.0, advect=0.0)):
        uhat = rng.standard_normal(fam.n)
        u, lam = project_sample(fam, uhat)
        A, _ = probe_affine(fam.h, fam.n)
        g = rng.standard_normal(fam.n)
        expect = g - A.T @ np.linalg.solve(A @ A.T, A @ g)
        np.testing.assert_allclose(adjoint_sample(fam, u, lam, g), expect, atol=1e-12)


@pytest.mark.parametrize("case", range(4))
def test_adjoint_symmetry_tangency_and_central_differences(case):
    fam, uhat = _all_tiny()[case]
    rng = np.random.default_rng(case)
    u, lam = project_sample(fam, uhat)
    v, w = rng.standard_normal(fam.n), rng.standard_normal(fam.n)
    Dv = adjoint_sample(fam, u, lam, v)
    Dw = adjoint_sample(fam, u, lam, w)
    # du*/du_hat = Z (Z^T W Z)^{-1} Z^T is symmetric
    assert abs(v @ Dw - w @ Dv) < 1e-10 * (1 + abs(v @ Dw))
    # the gradient lies in the tangent space of {h = 0}
    assert np.abs(fd_jac(fam.h, u) @ Dv).max() < 1e-7
    # central differences of the forward projection
    eps = 1e-6
    up, _ = project_sample(fam, uhat + eps * w)
    um, _ = project_sample(fam, uhat - eps * w)
    fd = v @ (up - um) / (2 * eps)
    assert abs(fd - v @ Dw) < 1e-6 * (1 + abs(fd))
