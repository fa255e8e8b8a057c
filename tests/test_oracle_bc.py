"""Pins of the oracle's Burgers boundary-row family (Dirichlet on the left,
Riemann-sum mass, one-sided Neumann on the right; paper Appendix A Burgers
problem, Appendix D discretizations) against facts that do not come from the
family's own formulas."""
import numpy as np
import pytest

import synthgen
from oracle.families import BurgersBC, family_of
from oracle.kkt import adjoint_sample, project_sample


def _grid(nx):
    return np.arange(nx) / (nx - 1)


def _affine(fam):
    """A and b of the linear rows h(u) = A u - b, probed by unit vectors."""
    h0 = fam.h(np.zeros(fam.n))
    A = np.stack([fam.h(np.eye(fam.n)[j]) - h0 for j in range(fam.n)], axis=1)
    return A, -h0


@pytest.mark.parametrize("nx,nt", [(3, 1), (5, 4), (12, 7)])
def test_projection_is_the_dense_affine_projection(nx, nt):
    rng = np.random.default_rng(nx * 10 + nt)
    fam = BurgersBC(nx, nt, 1.0 / (nx - 1), rng.uniform(), rng.uniform())
    uh = rng.standard_normal(fam.n)
    u, lam = project_sample(fam, uh)
    A, b = _affine(fam)
    expect = uh - A.T @ np.linalg.solve(A @ A.T, A @ uh - b)
    np.testing.assert_allclose(u, expect, rtol=0, atol=1e-12 * (1 + np.abs(expect).max()))
    # u = u_hat - A^T lam at the solution (the sign convention of the library)
    np.testing.assert_allclose(uh - A.T @ lam, u, rtol=0, atol=1e-11)


@pytest.mark.parametrize("nx", [11, 21, 41, 81, 161])
def test_rows_discretize_the_continuous_conditions(nx):
    # a smooth field on [0, 1] with u(0) = 5, u'(1) = 2 and integral 5 + 1/3:
    # the Dirichlet row is exact, the Neumann row tends to u'(1) (error
    # dx u''/2 = dx) and the mass row (with m0 = the integral) to 0 at first
    # order (the sum over both ends counts about dx (u(0) + u(1)) / 2 extra)
    x = _grid(nx)
    u = 5.0 + x * x
    fam = BurgersBC(nx, 1, 1.0 / (nx - 1), 5.0, 5.0 + 1.0 / 3.0)
    d, m, n = fam.h(u)
    dx = 1.0 / (nx - 1)
    assert abs(d) == 0.0
    assert abs(n - 2.0) <= 1.01 * dx
    assert abs(m) <= dx * np.abs(u).max()


def test_first_order_convergence_of_the_boundary_difference():
    errs = []
    for nx in (21, 41, 81):
        x = _grid(nx)
        fam = BurgersBC(nx, 1, 1.0 / (nx - 1), 0.0, 0.0)
        errs.append(abs(fam.h(np.sin(3.0 * x))[2] - 3.0 * np.cos(3.0)))
    assert 1.8 <= errs[0] / errs[1] <= 2.4 and 1.8 <= errs[1] / errs[2] <= 2.4, errs


def test_feasible_field_is_a_fixed_point():
    # build a field that meets the conditions by construction: left end at
    # u_L, last two values equal, interior shifted to the target mass
    rng = np.random.default_rng(3)
    nx, nt, uL, m0 = 17, 5, 0.4, 0.7
    dx = 1.0 / (nx - 1)
    U = rng.standard_normal((nt, nx))
    U[:, 0] = uL
    U[:, -1] = U[:, -2]
    for k in range(nt):
        # shift x = 1..nx-3 and the flat pair together keeps both conditions
        idx = np.arange(1, nx)
        U[k, idx] += (m0 / dx - U[k].sum()) / idx.size
    fam = BurgersBC(nx, nt, dx, uL, m0)
    assert np.abs(fam.h(U.reshape(-1))).max() <= 1e-12
    u, lam = project_sample(fam, U.reshape(-1))
    np.testing.assert_allclose(u, U.reshape(-1), rtol=0, atol=1e-13)
    assert np.abs(lam).max() <= 1e-11


def test_adjoint_is_the_null_space_projector():
    rng = np.random.default_rng(4)
    fam = BurgersBC(9, 3, 1.0 / 8, 0.2, 0.5)
    uh = rng.standard_normal(fam.n)
    u, lam = project_sample(fam, uh)
    g = rng.standard_normal(fam.n)
    A, _ = _affine(fam)
    P = np.eye(fam.n) - A.T @ np.linalg.solve(A @ A.T, A)
    np.testing.assert_allclose(adjoint_sample(fam, u, lam, g), P @ g, rtol=0, atol=1e-12)


def test_generated_batch_solves():
    b = synthgen.burgers_bc_batch(batch=2, nx=33, nt=9, seed=8)
    for smp in b.samples:
        fam = family_of(smp)
        u, lam = project_sample(fam, smp.uhat.reshape(-1))
        assert np.abs(fam.h(u)).max() <= 1e-11
