"""Pins of the oracle's SQP globalization and of its spectral form of the 2D
diffusion + energy family.

* Strongly nonlinear Fisher-KPP draws (dt*rho up to 1.1): the l1-merit SQP
  reaches a KKT point on every sample, and that point is a strict local
  minimizer (second-order sufficiency on null(J)).
* An independent solver (scipy SLSQP, a quasi-Newton SQP) reaches the same
  point on tiny grids.
* The real Fourier basis is orthonormal and diagonalizes the periodic second
  difference with the stated eigenvalues; the spectral form of the 2D family
  has the physical family's rows (rotated) and the same projection.
* The oracle refuses to return a point that is not a KKT point.
"""
import numpy as np
import pytest
from scipy.optimize import minimize

import synthgen
from oracle.families import Diff2DEnergySpectral, family_of, real_fourier_basis
from oracle.kkt import OracleNotConverged, project_sample, reduced_hessian_min_eig

STRONG = [(dt, seed) for dt in (0.45, 0.5, 0.55) for seed in range(1, 6)]


@pytest.mark.parametrize("dt,seed", STRONG)
def test_strongly_nonlinear_fisher_reaches_strict_minimizer(dt, seed):
    b = synthgen.fisher_kpp_batch(batch=4, nx=20, nt=8, seed=seed, dt=dt)
    for s in b.samples:
        fam = family_of(s)
        uhat = s.uhat.reshape(-1)
        u, lam, info = project_sample(fam, uhat, return_info=True)
        assert info["converged"]
        assert np.abs(fam.h(u)).max() <= 1e-12
        assert np.abs(u - uhat + fam.jac(u).T @ lam).max() <= 1e-12
        assert reduced_hessian_min_eig(fam, u, lam) > 1e-3


def _slsqp(fam, uhat):
    r = minimize(lambda x: 0.5 * np.sum((x - uhat) ** 2), uhat, jac=lambda x: x - uhat,
                 constraints=[{"type": "eq", "fun": fam.h, "jac": lambda x: fam.jac(x).toarray()}],
                 method="SLSQP", options=dict(maxiter=500, ftol=1e-16))
    return r.x


@pytest.mark.parametrize("seed,dt", [(1, 0.5), (4, 0.55), (2, 0.1)])
def test_fisher_agrees_with_slsqp(seed, dt):
    b = synthgen.fisher_kpp_batch(batch=3, nx=6, nt=4, seed=seed, dt=dt)
    for s in b.samples:
        fam = family_of(s)
        uhat = s.uhat.reshape(-1)
        u, _ = project_sample(fam, uhat)
        x = _slsqp(fam, uhat)
        assert np.abs(fam.h(x)).max() <= 1e-9
        assert np.linalg.norm(u - x) / np.linalg.norm(u) <= 1e-6


def test_diff2d_agrees_with_slsqp():
    b = synthgen.diff2d_batch(batch=3, n=6, nt=4, seed=41)
    for s in b.samples:
        fam = family_of(s)
        uhat = s.uhat.reshape(-1)
        u, lam = project_sample(fam, uhat, basis="physical")
        x = _slsqp(fam, uhat)
        assert np.abs(fam.h(x)).max() <= 1e-9
        assert np.linalg.norm(u - x) / np.linalg.norm(u) <= 1e-6
        assert reduced_hessian_min_eig(fam, u, lam) > 1e-3


@pytest.mark.parametrize("n", [4, 8, 64])
def test_real_fourier_basis_diagonalizes_periodic_second_difference(n):
    Q, f = real_fourier_basis(n)
    np.testing.assert_allclose(Q.T @ Q, np.eye(n), atol=1e-13)
    D = -2.0 * np.eye(n) + np.roll(np.eye(n), 1, axis=0) + np.roll(np.eye(n), -1, axis=0)
    np.testing.assert_allclose(Q.T @ D @ Q, np.diag(-4.0 * np.sin(np.pi * f / n) ** 2), atol=1e-12)


def test_spectral_diff2d_rows_are_rotated_physical_rows():
    s = synthgen.diff2d_batch(batch=1, n=16, nt=5, seed=7).samples[0]
    fam = family_of(s)
    sf = Diff2DEnergySpectral(fam)
    u = np.random.default_rng(2).standard_normal(fam.n)
    v = sf.to_spectral(u)
    np.testing.assert_allclose(sf.from_spectral(v), u, atol=1e-13)
    k = (fam.nt - 1) * fam.np_
    hs, hp = sf.h(v), fam.h(u)
    np.testing.assert_allclose(sf.from_spectral(hs[:k]), hp[:k], atol=1e-12)
    np.testing.assert_allclose(hs[k:], hp[k:], atol=1e-10)
    # Jacobian: J_spec = diag(Q^T, I) J_phys P, checked on a direction
    dv = np.random.default_rng(3).standard_normal(fam.n)
    lhs = sf.jac(v) @ dv
    rhs = fam.jac(u) @ sf.from_spectral(dv)
    np.testing.assert_allclose(sf.from_spectral(lhs[:k]), rhs[:k], atol=1e-11)
    np.testing.assert_allclose(lhs[k:], rhs[k:], atol=1e-10)


def test_spectral_and_physical_projection_agree():
    # two exact solves of the same problem in two orthonormal bases; the
    # agreement is limited by the conditioning of the energy rows
    for n, nt in ((8, 4), (12, 4)):
        b = synthgen.diff2d_batch(batch=2, n=n, nt=nt, seed=43)
        for s in b.samples:
            fam = family_of(s)
            uhat = s.uhat.reshape(-1)
            up, lp = project_sample(fam, uhat, basis="physical")
            us, ls = project_sample(fam, uhat)          # spectral route
            assert np.linalg.norm(us - up) / np.linalg.norm(up) <= 1e-9
            assert np.abs(fam.h(us)).max() <= 1e-10
            assert np.abs(us - uhat + fam.jac(us).T @ ls).max() <= 1e-9


def test_oracle_refuses_unconverged_points():
    s = synthgen.fisher_kpp_batch(batch=1, nx=20, nt=8, seed=4, dt=0.55).samples[0]
    fam = family_of(s)
    with pytest.raises(OracleNotConverged):
        project_sample(fam, s.uhat.reshape(-1), max_iter=2)
    u, lam, info = project_sample(fam, s.uhat.reshape(-1), max_iter=2, strict=False,
                                  return_info=True)
    assert not info["converged"]
