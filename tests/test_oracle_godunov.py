"""Pins of the oracle's Godunov-flux Burgers family (paper Appendix D,
Godunov's flux conservation) against facts fixed outside its own formulas:
Riemann-problem flux values, consistency with the PDE, finite differences,
and an independent solver on a tiny instance."""
import numpy as np
import pytest
from scipy.optimize import minimize

import synthgen
from oracle.families import BurgersGodunov, family_of
from oracle.kkt import project_sample


def _fd(fun, x, eps=1e-6):
    f0 = fun(x)
    out = np.empty((f0.size, x.size))
    for j in range(x.size):
        e = np.zeros_like(x)
        e[j] = eps
        out[:, j] = (fun(x + e) - fun(x - e)) / (2 * eps)
    return out


def test_riemann_problem_flux_values():
    F = lambda a, b: float(BurgersGodunov.flux(np.array([a]), np.array([b]))[0][0])
    assert F(1.0, -1.0) == 0.5          # stationary shock: both sides' flux
    assert F(-1.0, 1.0) == 0.0          # transonic expansion: f at the sonic point 0
    assert F(0.7, 0.3) == 0.5 * 0.7 ** 2    # both right-moving: upwind (left) state
    assert F(-0.2, -0.6) == 0.5 * 0.6 ** 2  # both left-moving: upwind (right) state
    assert F(0.9, -0.4) == 0.5 * 0.9 ** 2   # shock moving right: left state's flux
    assert F(0.3, -0.8) == 0.5 * 0.8 ** 2   # shock moving left: right state's flux


def test_residual_is_consistent_with_the_inviscid_pde():
    # smooth positive solution of u_t + u u_x = 0 near x = 0.5, found by the
    # characteristics u = u0(x - u t); the upwind-branch residual / dt -> 0
    def exact(x, t):
        u = np.full_like(x, 1.0)
        for _ in range(60):
            u = 1.0 + 0.2 * np.sin(2 * np.pi * (x - u * t))
        return u
    errs = []
    for nx in (64, 128, 256):
        dx = 1.0 / nx
        dt = 0.2 * dx
        x = np.arange(nx) * dx
        U = np.stack([exact(x, k * dt) for k in range(3)])
        fam = BurgersGodunov(nx, 3, dt, dx, 0.0)
        r = fam.h(U.reshape(-1)).reshape(2, nx) / dt
        errs.append(np.abs(r).max())
    assert errs[1] < errs[0] / 1.8 and errs[2] < errs[1] / 1.8, errs


def test_flux_differences_telescope():
    rng = np.random.default_rng(3)
    fam = BurgersGodunov(13, 4, 0.002, 1 / 13, 0.01)
    u = rng.standard_normal(fam.n)
    R = fam.h(u).reshape(3, 13)
    U = u.reshape(4, 13)
    np.testing.assert_allclose(R.sum(axis=1), U[1:].sum(axis=1) - U[:-1].sum(axis=1), atol=1e-12)


def test_ic_flux_and_mass_rows_are_rank_deficient():
    # The paper's Godunov regime stacks IC rows, flux-update rows and mass rows
    # m(t_k) - m(t_0).  IC and flux rows alone are Nx*Nt rows on Nx*Nt
    # unknowns and fix u; the mass rows add Nt-1 rows that are combinations of
    # them on a periodic grid, so the stacked Jacobian has rank Nx*Nt and
    # S = J J^T (W = I) is singular: the reason that regime is not projected.
    rng = np.random.default_rng(11)
    nx, nt = 7, 4
    fam = BurgersGodunov(nx, nt, 0.01, 1 / nx, 0.0)
    u = _away_from_kinks(fam, rng)
    ic = np.eye(fam.n)[:nx]
    mass = np.zeros((nt - 1, fam.n))
    for k in range(1, nt):
        mass[k - 1, k * nx:(k + 1) * nx] = fam.dx
        mass[k - 1, :nx] = -fam.dx
    jf = fam.jac(u).toarray()
    square = np.vstack([ic, jf])
    assert square.shape == (fam.n, fam.n) and np.linalg.matrix_rank(square) == fam.n
    stacked = np.vstack([ic, jf, mass])
    assert np.linalg.matrix_rank(stacked) == fam.n < stacked.shape[0]
    assert np.linalg.matrix_rank(stacked @ stacked.T) == fam.n


def _away_from_kinks(fam, rng, margin=0.05):
    # states with |u| > margin (away from the sonic point) and no interface
    # near a zero-speed shock (a > 0 > b with a = -b), where the branches tie
    for _ in range(10000):
        u = rng.uniform(-1.0, 1.0, fam.n)
        u = np.sign(u) * (margin + np.abs(u))
        U = u.reshape(fam.nt, fam.nx)
        a, b = U, np.roll(U, -1, axis=1)
        tie = (a > 0) & (b < 0) & (np.abs(a + b) < margin)
        if not tie.any():
            return u
    raise AssertionError("no draw away from the kinks")


def test_jacobian_and_hessian_against_finite_differences():
    rng = np.random.default_rng(7)
    fam = BurgersGodunov(9, 4, 0.01, 1 / 9, 0.005)
    u = _away_from_kinks(fam, rng)
    np.testing.assert_allclose(fam.jac(u).toarray(), _fd(fam.h, u), rtol=0, atol=1e-8)
    lam = rng.standard_normal(fam.m)
    grad = lambda v: fam.jac(v).T @ lam
    np.testing.assert_allclose(fam.hess(u, lam).toarray(), _fd(grad, u, 1e-6), rtol=0, atol=1e-6)


def test_independent_solver_agrees_on_a_tiny_instance():
    s = synthgen.godunov_batch(batch=1, nx=6, nt=3, dt=0.02, seed=5).samples[0]
    fam = family_of(s)
    uhat = s.uhat.reshape(-1)
    u, _ = project_sample(fam, uhat)
    res = minimize(lambda v: 0.5 * np.sum((v - uhat) ** 2), uhat, jac=lambda v: v - uhat,
                   constraints=[{"type": "eq", "fun": fam.h}], method="SLSQP",
                   options=dict(ftol=1e-15, maxiter=500))
    assert np.abs(fam.h(res.x)).max() < 1e-8
    np.testing.assert_allclose(u, res.x, atol=1e-6)


def test_generated_batches_converge():
    for seed in range(3):
        b = synthgen.godunov_batch(batch=3, nx=24, nt=12, seed=seed)
        for smp in b.samples:
            fam = family_of(smp)
            u, lam = project_sample(fam, smp.uhat.reshape(-1))
            assert np.abs(fam.h(u)).max() <= 1e-11
