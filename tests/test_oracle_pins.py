"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

None of these re-types the oracle's formulas: the checks use the printed
Appendix C matrix, closed forms computed a different way (dense linear algebra
on a constraint matrix probed from h), finite-difference Jacobians, an
independent SQP solver, PDE consistency on exact solutions, and invariants.
"""
import os

import numpy as np
import pytest
from scipy.optimize import minimize

import synthgen
from oracle.families import BurgersLF, Diff2DEnergy, FisherKPP, MassIC, family_of
from oracle.kkt import project_sample
from oracle.metric import constraint_error, max_violation

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def fd_jac(h, u, eps=1e-6):
    cols = []
    for j in range(u.size):
        e = np.zeros_like(u)
        e[j] = eps
        cols.append((h(u + e) - h(u - e)) / (2 * eps))
    return np.stack(cols, axis=1)


def probe_affine(h, n):
    """A, b with h(u) = A u - b, from evaluations of h only (h must be affine)."""
    h0 = h(np.zeros(n))
    A = np.stack([h(np.eye(n)[j]) - h0 for j in range(n)], axis=1)
    return A, -h0


def affine_projection(A, b, uhat):
    return uhat - A.T @ np.linalg.solve(A @ A.T, A @ uhat - b)


# ---------------------------------------------------------------- mass + IC

def test_appendix_c_jacobian_matches_printed_matrix():
    printed = np.loadtxt(os.path.join(GOLDEN, "appendix_c_jacobian.txt"))
    fam = MassIC(3, 3, g=np.array([0.3, -0.1, 0.7]), encoding="appendix_c")
    u = np.random.default_rng(0).standard_normal(9)
    assert fam.jac(u).toarray().shape == (5, 9)
    np.testing.assert_array_equal(fam.jac(u).toarray(), printed)


def test_mass_ic_elementwise_closed_form():
    # IC fixes slab 0; each later slab moves uniformly to hit the mass
    b = synthgen.mass_ic_batch(batch=3, nx=16, nt=6, seed=11)
    for s in b.samples:
        fam = family_of(s)
        u, lam = project_sample(fam, s.uhat.reshape(-1))
        U = u.reshape(s.nt, s.nx)
        g, m0 = s.aux[: s.nx], s.aux[s.nx]
        np.testing.assert_allclose(U[0], g, atol=1e-13)
        expect = s.uhat[1:] - ((s.uhat[1:].sum(axis=1) - m0) / s.nx)[:, None]
        np.testing.assert_allclose(U[1:], expect, atol=1e-12)
        # multipliers: IC rows u_hat(.,0) - g; mass rows (sum u_hat - M0)/Nx
        np.testing.assert_allclose(lam[: s.nx], s.uhat[0] - g, atol=1e-12)
        np.testing.assert_allclose(lam[s.nx:], (s.uhat[1:].sum(axis=1) - m0) / s.nx, atol=1e-12)


def test_mass_encodings_give_same_field():
    # row scaling and "relative to the IC slab" change lam, never u
    rng = np.random.default_rng(3)
    nx, nt = 7, 5
    g = rng.standard_normal(nx)
    uhat = rng.standard_normal(nx * nt)
    base = MassIC(nx, nt, g)
    u0, _ = project_sample(base, uhat)

    class Scaled(MassIC):
        def h(self, u):
            r = super().h(u)
            r[self.nx:] *= 1.0 / self.nx        # Riemann sum with dx
            return r

        def jac(self, u):
            J = super().jac(u).tolil()
            J[self.nx:, :] = J[self.nx:, :] / self.nx
            return J.tocsr()

    u1, _ = project_sample(Scaled(nx, nt, g), uhat)
    np.testing.assert_allclose(u1, u0, atol=1e-12)


def test_linear_families_equal_dense_affine_projection():
    rng = np.random.default_rng(5)
    cases = [
        MassIC(6, 4, rng.standard_normal(6)),
        FisherKPP(6, 4, rng.uniform(0.2, 0.8, 6), rho=0.0, dt=0.1),
        BurgersLF(6, 4, dt=0.01, dx=1 / 6, nu=0.01, alpha=1.0, advect=0.0),
    ]
    for fam in cases:
        uhat = rng.standard_normal(fam.n)
        A, bb = probe_affine(fam.h, fam.n)
        expect = affine_projection(A, bb, uhat)
        u, lam = project_sample(fam, uhat)
        np.testing.assert_allclose(u, expect, atol=1e-12)
        # lam = (A A^T)^{-1} (A u_hat - b)
        np.testing.assert_allclose(lam, np.linalg.solve(A @ A.T, A @ uhat - bb), atol=1e-11)


# ---------------------------------------------------------------- Fisher-KPP

def test_fisher_logistic_trajectory_is_feasible():
    # spatially uniform explicit-Euler logistic growth conserves the discrete budget
    nx, nt, rho, dt = 8, 6, 1.3, 0.05
    v = [0.2]
    for _ in range(nt - 1):
        v.append(v[-1] + dt * rho * v[-1] * (1 - v[-1]))
    U = np.repeat(np.array(v)[:, None], nx, axis=1)
    fam = FisherKPP(nx, nt, g=U[0], rho=rho, dt=dt)
    assert np.abs(fam.h(U.reshape(-1))).max() < 1e-13


def test_fisher_two_steps_is_a_hyperplane_projection():
    # Nt = 2: the IC pins slab 0, so slab 1 is projected onto one hyperplane
    rng = np.random.default_rng(9)
    nx, rho, dt = 9, 1.7, 0.2
    g = rng.uniform(0.1, 0.9, nx)
    uhat = rng.uniform(0, 1, 2 * nx)
    fam = FisherKPP(nx, 2, g, rho, dt)
    u, _ = project_sample(fam, uhat)
    target = g.sum() + dt * rho * (g * (1 - g)).sum()
    u1 = uhat[nx:] - (uhat[nx:].sum() - target) / nx
    np.testing.assert_allclose(u[:nx], g, atol=1e-13)
    np.testing.assert_allclose(u[nx:], u1, atol=1e-12)


# ---------------------------------------------------------------- Burgers

def _taylor_wave(x, t, amp, speed, nu_eff, x0=0.5):
    return speed - amp * np.tanh(amp * (x - x0 - speed * t) / (2 * nu_eff))


@pytest.mark.parametrize("nu,alpha", [(0.01, 0.1), (0.02, 0.0)])
def test_burgers_residual_is_consistent_with_the_pde(nu, alpha):
    # exact travelling wave of u_t + u u_x = nu_eff u_xx, nu_eff = nu + alpha dx/2
    errs = []
    for nx in (64, 128, 256):
        dx = 1.0 / nx
        dt = 0.1 * dx
        nu_eff = nu + 0.5 * alpha * dx
        x = np.arange(nx) * dx
        U = np.stack([_taylor_wave(x, k * dt, 0.5, 0.3, nu_eff) for k in range(3)])
        fam = BurgersLF(nx, 3, dt, dx, nu, alpha)
        r = fam.h(U.reshape(-1)).reshape(2, nx) / dt
        interior = (x > 0.2) & (x < 0.8)
        errs.append(np.abs(r[:, interior]).max())
    assert errs[1] < errs[0] / 2.5 and errs[2] < errs[1] / 2.5, errs


def test_burgers_flux_differences_telescope():
    # sum_i R_{k,i} = sum_i u^{k+1} - sum_i u^k on a periodic grid
    rng = np.random.default_rng(2)
    fam = BurgersLF(11, 5, 0.003, 1 / 11, 0.02, 0.7)
    u = rng.standard_normal(fam.n)
    R = fam.h(u).reshape(4, 11)
    U = u.reshape(5, 11)
    np.testing.assert_allclose(R.sum(axis=1), U[1:].sum(axis=1) - U[:-1].sum(axis=1), atol=1e-12)


def test_burgers_feasible_input_is_a_fixed_point():
    b = synthgen.burgers_batch(batch=1, nx=16, nt=8, seed=4)
    s = b.samples[0]
    fam = family_of(s)
    # rebuild the noise-free trajectory from the first slab, by solving h = 0 slab by slab
    U = s.uhat.copy()
    for k in range(s.nt - 1):
        r = fam.h(U.reshape(-1)).reshape(s.nt - 1, s.nx)[k]
        U[k + 1] -= r                                   # dR_k/du^{k+1} = I
    clean = U.reshape(-1)
    assert np.abs(fam.h(clean)).max() < 1e-14
    u, lam = project_sample(fam, clean)
    np.testing.assert_allclose(u, clean, atol=1e-14)
    assert np.abs(lam).max() < 1e-13


# ---------------------------------------------------------------- 2D diffusion + energy

def test_diff2d_residual_is_consistent_with_heat_equation():
    errs = []
    for n in (8, 16, 32):
        dx = 1.0 / n
        dt = 0.2 * dx * dx
        kappa = 0.05
        x = np.arange(n) * dx
        X, Y = np.meshgrid(x, x, indexing="xy")
        rate = kappa * (2 * np.pi) ** 2 * 2
        U = np.stack([np.exp(-rate * k * dt) * np.cos(2 * np.pi * (X + Y)) for k in range(2)])
        fam = Diff2DEnergy(n, n, 2, dt, dx, kappa, energy=np.zeros(2))
        r = fam.split(fam.h(U.reshape(-1)))["residual"] / dt
        errs.append(np.abs(r).max())
    assert errs[1] < errs[0] / 3 and errs[2] < errs[1] / 3, errs


def test_single_energy_row_is_a_sphere_projection():
    rng = np.random.default_rng(8)
    n = 5
    uhat = rng.standard_normal(n * n)
    E = 3.7
    fam = Diff2DEnergy(n, n, 1, 0.01, 0.2, 0.05, energy=np.array([E]))
    u, lam = project_sample(fam, uhat)
    r = np.linalg.norm(uhat)
    np.testing.assert_allclose(u, np.sqrt(E) * uhat / r, atol=1e-13)
    np.testing.assert_allclose(lam[0], (r / np.sqrt(E) - 1) / 2, atol=1e-13)


# ---------------------------------------------------------------- all families

def _tiny_samples():
    return [
        synthgen.mass_ic_batch(batch=1, nx=5, nt=4, seed=1).samples[0],
        synthgen.fisher_kpp_batch(batch=1, nx=6, nt=4, seed=2).samples[0],
        synthgen.burgers_batch(batch=1, nx=6, nt=4, seed=3).samples[0],
    ]


def _tiny_2d():
    s = synthgen.diff2d_batch(batch=1, n=4, nt=2, seed=4).samples[0]
    # a stronger diffusion number keeps the two energy rows well separated;
    # targets come from a trajectory made feasible for the residual rows
    kappa = 2.0
    probe = Diff2DEnergy(4, 4, 2, s.dt, s.dx, kappa, np.zeros(2))
    nres = 16
    A, b = probe_affine(lambda v: probe.h(v)[:nres], probe.n)
    clean = affine_projection(A, b, s.uhat.reshape(-1))
    energy = (clean.reshape(2, -1) ** 2).sum(axis=1)
    fam = Diff2DEnergy(4, 4, 2, s.dt, s.dx, kappa, energy)
    noise = 0.05 * np.random.default_rng(1).standard_normal(probe.n)
    return fam, clean + noise


def _all_tiny():
    out = [(family_of(s), s.uhat.reshape(-1)) for s in _tiny_samples()]
    out.append(_tiny_2d())
    return out


@pytest.mark.parametrize("case", range(4))
def test_kkt_conditions_with_finite_difference_jacobian(case):
    fam, uhat = _all_tiny()[case]
    u, lam = project_sample(fam, uhat)
    Jfd = fd_jac(fam.h, u)
    assert np.abs(fam.h(u)).max() < 1e-12
    assert np.abs(u - uhat + Jfd.T @ lam).max() < 1e-7
    # second-order sufficiency on null(J): Z^T W Z > 0, W from FD of the Lagrangian gradient
    grad = lambda v: v - uhat + fd_jac(fam.h, v).T @ lam
    W = fd_jac(grad, u, eps=1e-4)
    _, sv, vt = np.linalg.svd(Jfd)
    rank = int((sv > 1e-9 * sv[0]).sum())
    Z = vt[rank:].T
    if Z.shape[1]:
        assert np.linalg.eigvalsh(Z.T @ (0.5 * (W + W.T)) @ Z).min() > 0


@pytest.mark.parametrize("case", range(4))
def test_independent_sqp_solver_agrees(case):
    fam, uhat = _all_tiny()[case]
    u, _ = project_sample(fam, uhat)
    res = minimize(lambda v: 0.5 * np.sum((v - uhat) ** 2), uhat, jac=lambda v: v - uhat,
                   constraints=[{"type": "eq", "fun": fam.h}], method="SLSQP",
                   options=dict(ftol=1e-15, maxiter=500))
    assert np.abs(fam.h(res.x)).max() < 1e-8
    np.testing.assert_allclose(u, res.x, atol=1e-6)


@pytest.mark.parametrize("case", range(4))
def test_projection_is_idempotent(case):
    fam, uhat = _all_tiny()[case]
    u, _ = project_sample(fam, uhat)
    u2, lam2 = project_sample(fam, u)
    np.testing.assert_allclose(u2, u, atol=1e-12)
    assert np.abs(lam2).max() < 1e-10


def test_batch_samples_are_independent():
    b = synthgen.fisher_kpp_batch(batch=3, nx=8, nt=5, seed=21)
    b1 = synthgen.Batch([b.samples[1]]).pack()
    from oracle.kkt import project_batch
    u3, lam3, _ = project_batch(b)
    u1, lam1, _ = project_batch(b1)
    np.testing.assert_array_equal(u3[b.var_off[1]: b.var_off[1] + b.samples[1].n], u1)
    np.testing.assert_array_equal(lam3[b.row_off[1]: b.row_off[1] + b.samples[1].m], lam1)


def test_constraint_error_metric_on_hand_example():
    b = synthgen.mass_ic_batch(batch=2, nx=3, nt=2, seed=0)
    u = b.uhat.copy()
    errs = constraint_error(b, u)
    expect_ic, expect_mass = [], []
    for s in b.samples:
        g, m0 = s.aux[:3], s.aux[3]
        expect_ic.append(np.sqrt(((s.uhat[0] - g) ** 2).sum()))
        expect_mass.append(abs(s.uhat[1].sum() - m0))
    assert errs["ic"] == pytest.approx(np.mean(expect_ic))
    assert errs["mass"] == pytest.approx(np.mean(expect_mass))
    mv = max_violation(b, u)
    assert mv[0] == pytest.approx(max(np.abs(b.samples[0].uhat[0] - b.samples[0].aux[:3]).max(),
                                      expect_mass[0]))
