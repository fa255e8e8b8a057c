"""Constraint families of the oracle: h(u), J(u), Hessian of lam^T h.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Variables of one sample are the discretized field flattened time-slab major,
x fastest (2D: slab, then y, then x), as in the paper's worked Jacobian
example (Appendix C).  Rows are in the canonical order documented per family;
the GPU library returns its multipliers in the same order.

Every function here is the definition written out with numpy/scipy.sparse;
none of it is shared with the GPU code.

Pins (tests/test_oracle_pins.py):
  mass_ic     Appendix C printed 5x9 Jacobian; elementwise closed form.
  fisher_kpp  logistic explicit-Euler trajectories are feasible; rho = 0 and
              Nt = 2 reduce to closed-form hyperplane projections; J and the
              Hessian against finite differences of h.
  burgers_lf  consistency of the residual with the viscous Burgers PDE on an
              exact travelling wave (residual/dt -> 0 under refinement);
              telescoping of the flux differences; J and Hessian vs FD.
  diff2d      consistency with the heat equation on a decaying Fourier mode;
              single energy row = sphere projection (closed form); J/Hessian
              vs FD.
  godunov     an exact steady shock and the sonic expansion give the
              flux values Riemann's problem fixes; consistency with the
              inviscid PDE on a smooth one-signed wave; J and the Hessian vs
              finite differences away from the flux's kinks.
  burgers_bc  dense affine projection (closed form); a discrete field built to
              meet the boundary conditions and the mass is a fixed point; the
              Neumann row vanishes on fields flat at the right end and the
              Dirichlet row reads the left end only.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

MASS_IC, FISHER_KPP, BURGERS_LF, DIFF2D_ENERGY, BURGERS_BC, BURGERS_GODUNOV = 1, 2, 3, 4, 5, 6


def _vid1(nx, k, i):
    """flat index of u(x_i, t_k) in a 1D sample"""
    return k * nx + i


class MassIC:
    """Initial condition + per-step mass (paper Table 1 rows 'Dirichlet IC' and
    'Global mass conservation'; Heat-1 constraint set, Appendix A; Appendix C).

    Canonical rows:
      IC rows   u(x_i, t_0) - g_i                      i = 0..Nx-1
      mass rows sum_i u(x_i, t_k) - M0                 k = 1..Nt-1
    The t_0 mass row is left out (Appendix C omits the first-step mass row);
    with the IC rows present it would be the sum of the IC rows.

    encoding='appendix_c' gives the exact rows of the Appendix C example:
      mass rows sum_{i < Nx-1} u(x_i, t_k) - sum_{i < Nx-1} u(x_i, t_0)
    (left Riemann sum over the first Nx-1 points, relative to the first step).
    """
    types = ("ic", "mass")

    def __init__(self, nx, nt, g, m0=None, encoding="plain"):
        self.nx, self.nt = int(nx), int(nt)
        self.g = np.asarray(g, dtype=np.float64)
        self.m0 = float(self.g.sum() if m0 is None else m0)
        self.encoding = encoding
        self.n = self.nx * self.nt
        self.m = self.nx + self.nt - 1

    def h(self, u):
        U = u.reshape(self.nt, self.nx)
        ic = U[0] - self.g
        if self.encoding == "appendix_c":
            mass = U[1:, : self.nx - 1].sum(axis=1) - U[0, : self.nx - 1].sum()
        else:
            mass = U[1:].sum(axis=1) - self.m0
        return np.concatenate([ic, mass])

    def jac(self, u):
        rows, cols, vals = [], [], []
        for i in range(self.nx):
            rows.append(i); cols.append(_vid1(self.nx, 0, i)); vals.append(1.0)
        for k in range(1, self.nt):
            r = self.nx + k - 1
            if self.encoding == "appendix_c":
                for i in range(self.nx - 1):
                    rows.append(r); cols.append(_vid1(self.nx, k, i)); vals.append(1.0)
                    rows.append(r); cols.append(_vid1(self.nx, 0, i)); vals.append(-1.0)
            else:
                for i in range(self.nx):
                    rows.append(r); cols.append(_vid1(self.nx, k, i)); vals.append(1.0)
        return sp.csr_matrix((vals, (rows, cols)), shape=(self.m, self.n))

    def hess(self, u, lam):
        return sp.csr_matrix((self.n, self.n))

    def split(self, r):
        return {"ic": r[: self.nx], "mass": r[self.nx:]}


class FisherKPP:
    """Initial condition + nonlinear mass budget of the logistic reaction
    rho*u*(1-u) (paper Table 1 'Nonlinear conservation law'; reaction-diffusion
    constraint set, Appendix A; time-discretized as in Appendix D, forward
    difference in time of the spatial Riemann sum).  Periodic x, so no
    boundary-flux term.

    Canonical rows:
      IC rows   u(x_i, t_0) - g_i                                        i = 0..Nx-1
      law rows  sum_i u_i^{k+1} - sum_i u_i^k - dt*rho*sum_i u_i^k (1 - u_i^k)
                                                                       k = 0..Nt-2
    (The Appendix D form divides by dt and multiplies by dx; a row scaling
    changes the multipliers, never the projected field.)
    """
    types = ("ic", "law")

    def __init__(self, nx, nt, g, rho, dt):
        self.nx, self.nt = int(nx), int(nt)
        self.g = np.asarray(g, dtype=np.float64)
        self.rho, self.dt = float(rho), float(dt)
        self.n = self.nx * self.nt
        self.m = self.nx + self.nt - 1

    def h(self, u):
        U = u.reshape(self.nt, self.nx)
        ic = U[0] - self.g
        mass = U.sum(axis=1)
        react = (U * (1.0 - U)).sum(axis=1)
        law = mass[1:] - mass[:-1] - self.dt * self.rho * react[:-1]
        return np.concatenate([ic, law])

    def jac(self, u):
        U = u.reshape(self.nt, self.nx)
        nx, nt = self.nx, self.nt
        c = self.dt * self.rho
        i = np.arange(nx)
        k = np.arange(nt - 1)
        K, I = np.meshgrid(k, i, indexing="ij")              # (nt-1, nx)
        ic_r, ic_c, ic_v = i, _vid1(nx, 0, i), np.ones(nx)
        # +1 on slab k+1
        a_r, a_c, a_v = nx + K, _vid1(nx, K + 1, I), np.ones_like(K, dtype=float)
        # -1 - dt*rho*(1 - 2u) on slab k
        b_r, b_c = nx + K, _vid1(nx, K, I)
        b_v = -1.0 - c * (1.0 - 2.0 * U[:-1])
        rows = np.concatenate([ic_r, a_r.ravel(), b_r.ravel()])
        cols = np.concatenate([ic_c, a_c.ravel(), b_c.ravel()])
        vals = np.concatenate([ic_v, a_v.ravel(), b_v.ravel()])
        return sp.csr_matrix((vals, (rows, cols)), shape=(self.m, self.n))

    def hess(self, u, lam):
        lam_law = np.asarray(lam[self.nx:])
        d = np.zeros((self.nt, self.nx))
        # d^2/du^2 of -dt*rho*u*(1-u) is +2*dt*rho on slab k of law row k
        d[: self.nt - 1, :] = (2.0 * self.dt * self.rho * lam_law)[:, None]
        return sp.diags(d.reshape(-1))

    def split(self, r):
        return {"ic": r[: self.nx], "law": r[self.nx:]}


class BurgersLF:
    """Local flux-update residuals of viscous Burgers u_t + (u^2/2)_x = nu*u_xx
    on a periodic grid (paper Appendix D 'flux conservation': the residual is
    the mismatch between consecutive steps and one conservative finite-volume
    update; here with the smooth Lax-Friedrichs interface flux in place of the
    Godunov flux, plus a centred viscous term).

    Interface flux  F_{i+1/2} = (f(u_i) + f(u_{i+1}))/2 - (alpha/2)(u_{i+1} - u_i),
    f(u) = u^2/2.  Canonical rows, k-major, for k = 0..Nt-2 and i = 0..Nx-1:
      R_{k,i} = u_i^{k+1} - [ u_i^k - (dt/dx)(F_{i+1/2} - F_{i-1/2})
                              + nu*dt*(u_{i+1} - 2u_i + u_{i-1})/dx^2 ]   (all at step k)
    """
    types = ("flux",)

    def __init__(self, nx, nt, dt, dx, nu, alpha, advect=1.0):
        self.nx, self.nt = int(nx), int(nt)
        self.dt, self.dx, self.nu, self.alpha = float(dt), float(dx), float(nu), float(alpha)
        # f(u) = advect * u^2 / 2; advect = 0 leaves the linear viscous scheme
        self.advect = float(advect)
        self.n = self.nx * self.nt
        self.m = self.nx * (self.nt - 1)

    def _flux(self, a, b):
        return 0.25 * self.advect * (a * a + b * b) - 0.5 * self.alpha * (b - a)

    def h(self, u):
        U = u.reshape(self.nt, self.nx)
        out = np.empty((self.nt - 1, self.nx))
        r = self.dt / self.dx
        v = self.nu * self.dt / (self.dx * self.dx)
        for k in range(self.nt - 1):
            uk = U[k]
            up = np.roll(uk, -1)
            um = np.roll(uk, 1)
            Fp = self._flux(uk, up)       # F_{i+1/2}
            Fm = self._flux(um, uk)       # F_{i-1/2}
            update = uk - r * (Fp - Fm) + v * (up - 2.0 * uk + um)
            out[k] = U[k + 1] - update
        return out.reshape(-1)

    def jac(self, u):
        U = u.reshape(self.nt, self.nx)
        r = self.dt / self.dx
        v = self.nu * self.dt / (self.dx * self.dx)
        a = self.alpha
        nx, nt = self.nx, self.nt
        K, I = np.meshgrid(np.arange(nt - 1), np.arange(nx), indexing="ij")
        row = K * nx + I
        ip, im = (I + 1) % nx, (I - 1) % nx
        parts = [
            # d/du_i^{k+1}
            (row, _vid1(nx, K + 1, I), np.ones_like(row, dtype=float)),
            # d/du_i^k: dF_{i+1/2}/du_i = u_i/2 + a/2, dF_{i-1/2}/du_i = u_i/2 - a/2
            (row, _vid1(nx, K, I), np.full(row.shape, -1.0 + r * a + 2.0 * v)),
            # d/du_{i+1}^k: r*dF_{i+1/2}/du_{i+1} - v = r*(u_{i+1}/2 - a/2) - v
            (row, _vid1(nx, K, ip), r * (0.5 * self.advect * U[K, ip] - 0.5 * a) - v),
            # d/du_{i-1}^k: -r*dF_{i-1/2}/du_{i-1} - v = -r*(u_{i-1}/2 + a/2) - v
            (row, _vid1(nx, K, im), -r * (0.5 * self.advect * U[K, im] + 0.5 * a) - v),
        ]
        rows = np.concatenate([p[0].ravel() for p in parts])
        cols = np.concatenate([p[1].ravel() for p in parts])
        vals = np.concatenate([p[2].ravel() for p in parts])
        return sp.csr_matrix((vals, (rows, cols)), shape=(self.m, self.n))

    def hess(self, u, lam):
        L = np.asarray(lam).reshape(self.nt - 1, self.nx)
        half_r = 0.5 * self.advect * self.dt / self.dx
        d = np.zeros((self.nt, self.nx))
        for k in range(self.nt - 1):
            # row (k,i) has +half_r*u_{i+1}^2/... : second derivative +half_r at i+1,
            # -half_r at i-1
            d[k] += half_r * np.roll(L[k], 1)     # lam_{k,j-1} at position j
            d[k] -= half_r * np.roll(L[k], -1)    # lam_{k,j+1} at position j
        return sp.diags(d.reshape(-1))

    def split(self, r):
        return {"flux": r}


class Diff2DEnergy:
    """2D periodic diffusion with a per-frame quadratic invariant (Navier-Stokes
    analogue of Appendix A: local PDE residual rows as in the heat problem's
    'u_t - alpha*u_xx' rows, and an enstrophy-type row int w^2 - const per
    frame).

    Grid: Nx x Ny periodic with spacing dx in both directions, 5-point
    Laplacian Lap.  Canonical rows:
      residual rows  u^{k+1}(p) - u^k(p) - dt*kappa*(Lap u^{k+1})(p)
                     k = 0..Nt-2, p = (y, x) with x fastest
      energy rows    sum_p u^t(p)^2 - E_t                          t = 0..Nt-1
    """
    types = ("residual", "energy")

    def __init__(self, nx, ny, nt, dt, dx, kappa, energy):
        self.nx, self.ny, self.nt = int(nx), int(ny), int(nt)
        self.dt, self.dx, self.kappa = float(dt), float(dx), float(kappa)
        self.E = np.asarray(energy, dtype=np.float64)
        self.np_ = self.nx * self.ny
        self.n = self.np_ * self.nt
        self.m = (self.nt - 1) * self.np_ + self.nt

    def _lap(self, f):
        return (np.roll(f, 1, axis=0) + np.roll(f, -1, axis=0) + np.roll(f, 1, axis=1)
                + np.roll(f, -1, axis=1) - 4.0 * f) / (self.dx * self.dx)

    def h(self, u):
        U = u.reshape(self.nt, self.ny, self.nx)
        res = np.empty((self.nt - 1, self.ny, self.nx))
        for k in range(self.nt - 1):
            res[k] = U[k + 1] - U[k] - self.dt * self.kappa * self._lap(U[k + 1])
        energy = (U * U).reshape(self.nt, -1).sum(axis=1) - self.E
        return np.concatenate([res.reshape(-1), energy])

    def jac(self, u):
        U = u.reshape(self.nt, self.ny, self.nx)
        nx, ny, npt, nt = self.nx, self.ny, self.np_, self.nt
        s = self.dt * self.kappa / (self.dx * self.dx)
        K, Y, X = np.meshgrid(np.arange(nt - 1), np.arange(ny), np.arange(nx), indexing="ij")
        row = K * npt + Y * nx + X
        nxt = (K + 1) * npt
        parts = [(row, nxt + Y * nx + X, np.full(row.shape, 1.0 + 4.0 * s))]
        for (yy, xx) in (((Y + 1) % ny, X), ((Y - 1) % ny, X), (Y, (X + 1) % nx), (Y, (X - 1) % nx)):
            parts.append((row, nxt + yy * nx + xx, np.full(row.shape, -s)))
        parts.append((row, K * npt + Y * nx + X, np.full(row.shape, -1.0)))
        T, P = np.meshgrid(np.arange(nt), np.arange(npt), indexing="ij")
        parts.append(((nt - 1) * npt + T, T * npt + P, 2.0 * U.reshape(nt, npt)))
        rows = np.concatenate([p[0].ravel() for p in parts])
        cols = np.concatenate([p[1].ravel() for p in parts])
        vals = np.concatenate([p[2].ravel() for p in parts])
        return sp.csr_matrix((vals, (rows, cols)), shape=(self.m, self.n))

    def hess(self, u, lam):
        lam_e = np.asarray(lam[(self.nt - 1) * self.np_:])
        d = np.repeat(2.0 * lam_e, self.np_)
        return sp.diags(d)

    def split(self, r):
        k = (self.nt - 1) * self.np_
        return {"residual": r[:k], "energy": r[k:]}


class BurgersGodunov:
    """Local flux-update residuals of Burgers u_t + (u^2/2)_x = nu*u_xx on a
    periodic grid with Godunov's interface flux (paper Appendix D, Godunov's
    flux conservation: each row is the mismatch between consecutive steps and
    one conservative finite-volume update), plus a centred viscous term
    (nu = 0: the inviscid equation of the paper's Burgers problem).

    Godunov flux of the convex f(u) = u^2/2 (minimum at 0) between a left
    state a and a right state b:  F(a, b) = max(f(max(a, 0)), f(min(b, 0))).
    It is piecewise smooth; Newton steps use the derivative of the branch that
    attains the max (ties: the left state's branch), which is what makes the
    iteration a semismooth Newton method.  Canonical rows, k-major, for
    k = 0..Nt-2 and i = 0..Nx-1:
      R_{k,i} = u_i^{k+1} - [ u_i^k - (dt/dx)(F_{i+1/2} - F_{i-1/2})
                              + nu*dt*(u_{i+1} - 2u_i + u_{i-1})/dx^2 ]   (all at step k)
    """
    types = ("flux",)

    def __init__(self, nx, nt, dt, dx, nu):
        self.nx, self.nt = int(nx), int(nt)
        self.dt, self.dx, self.nu = float(dt), float(dx), float(nu)
        self.n = self.nx * self.nt
        self.m = self.nx * (self.nt - 1)

    @staticmethod
    def flux(a, b):
        """F, dF/da, dF/db, d2F/da2, d2F/db2 of Godunov's flux (elementwise)."""
        ap, bm = np.maximum(a, 0.0), np.minimum(b, 0.0)
        left = ap * ap >= bm * bm
        F = np.where(left, 0.5 * ap * ap, 0.5 * bm * bm)
        Fa = np.where(left, ap, 0.0)
        Fb = np.where(left, 0.0, bm)
        Faa = np.where(left & (a > 0.0), 1.0, 0.0)
        Fbb = np.where(~left & (b < 0.0), 1.0, 0.0)
        return F, Fa, Fb, Faa, Fbb

    def h(self, u):
        U = u.reshape(self.nt, self.nx)
        r = self.dt / self.dx
        v = self.nu * self.dt / (self.dx * self.dx)
        out = np.empty((self.nt - 1, self.nx))
        for k in range(self.nt - 1):
            uk = U[k]
            up, um = np.roll(uk, -1), np.roll(uk, 1)
            Fp = self.flux(uk, up)[0]
            Fm = self.flux(um, uk)[0]
            out[k] = U[k + 1] - (uk - r * (Fp - Fm) + v * (up - 2.0 * uk + um))
        return out.reshape(-1)

    def jac(self, u):
        U = u.reshape(self.nt, self.nx)
        r = self.dt / self.dx
        v = self.nu * self.dt / (self.dx * self.dx)
        nx, nt = self.nx, self.nt
        K, I = np.meshgrid(np.arange(nt - 1), np.arange(nx), indexing="ij")
        row = K * nx + I
        ip, im = (I + 1) % nx, (I - 1) % nx
        _, Fa_p, Fb_p, _, _ = self.flux(U[K, I], U[K, ip])    # interface i+1/2
        _, Fa_m, Fb_m, _, _ = self.flux(U[K, im], U[K, I])    # interface i-1/2
        parts = [
            (row, _vid1(nx, K + 1, I), np.ones_like(row, dtype=float)),
            (row, _vid1(nx, K, I), -1.0 + r * (Fa_p - Fb_m) + 2.0 * v),
            (row, _vid1(nx, K, ip), r * Fb_p - v),
            (row, _vid1(nx, K, im), -r * Fa_m - v),
        ]
        rows = np.concatenate([p[0].ravel() for p in parts])
        cols = np.concatenate([p[1].ravel() for p in parts])
        vals = np.concatenate([p[2].ravel() for p in parts])
        return sp.csr_matrix((vals, (rows, cols)), shape=(self.m, self.n))

    def hess(self, u, lam):
        # lam^T h: row (k, i) carries r*(F_{i+1/2} - F_{i-1/2}); each branch is
        # a square of one state, so the Hessian is diagonal
        U = u.reshape(self.nt, self.nx)
        L = np.asarray(lam).reshape(self.nt - 1, self.nx)
        r = self.dt / self.dx
        d = np.zeros((self.nt, self.nx))
        for k in range(self.nt - 1):
            uk = U[k]
            _, _, _, Faa_p, _ = self.flux(uk, np.roll(uk, -1))          # F(u_j, u_{j+1})
            _, _, _, _, Fbb_m = self.flux(np.roll(uk, 1), uk)          # F(u_{j-1}, u_j)
            # u_j enters F_{j+1/2} of rows j (+) and j+1 (-) as the left
            # state, F_{j-1/2} of rows j (-) and j-1 (+) as the right state
            d[k] = r * (Faa_p * (L[k] - np.roll(L[k], -1)) + Fbb_m * (np.roll(L[k], 1) - L[k]))
        return sp.diags(d.reshape(-1))

    def split(self, r):
        return {"flux": r}


class BurgersBC:
    """Boundary rows and global mass of the paper's first Burgers constraint
    regime (Appendix A, Burgers problem: the Dirichlet condition on the left
    boundary, the mass constraint and the Neumann condition on the right
    boundary), discretized as in Appendix D: the mass by the Riemann sum
    m(t_k) = sum_i u_i^k dx, the Neumann condition by the one-sided difference
    (u_{Nx-1}^k - u_{Nx-2}^k) / dx at the right end.  Grid x_i = i dx on
    [0, 1], i = 0..Nx-1, dx = 1 / (Nx - 1); one row of each kind per time step
    k = 0..Nt-1.

    Canonical rows (by kind, then step):
      Dirichlet  u_0^k - u_L                          k = 0..Nt-1
      mass       dx sum_i u_i^k - m0                  k = 0..Nt-1
      Neumann    (u_{Nx-1}^k - u_{Nx-2}^k) / dx       k = 0..Nt-1
    All rows are linear: the Hessian of lam^T h is zero.  Nx >= 3 keeps the
    three rows of a step independent.
    """
    types = ("dirichlet", "mass", "neumann")

    def __init__(self, nx, nt, dx, u_left, m0):
        self.nx, self.nt = int(nx), int(nt)
        if self.nx < 3:
            raise ValueError("Burgers boundary rows need nx >= 3")
        self.dx = float(dx)
        self.u_left, self.m0 = float(u_left), float(m0)
        self.n = self.nx * self.nt
        self.m = 3 * self.nt

    def h(self, u):
        U = u.reshape(self.nt, self.nx)
        dirichlet = U[:, 0] - self.u_left
        mass = self.dx * U.sum(axis=1) - self.m0
        neumann = (U[:, -1] - U[:, -2]) / self.dx
        return np.concatenate([dirichlet, mass, neumann])

    def jac(self, u):
        rows, cols, vals = [], [], []
        nt, nx = self.nt, self.nx
        for k in range(nt):
            rows.append(k); cols.append(_vid1(nx, k, 0)); vals.append(1.0)
            for i in range(nx):
                rows.append(nt + k); cols.append(_vid1(nx, k, i)); vals.append(self.dx)
            rows.append(2 * nt + k); cols.append(_vid1(nx, k, nx - 1)); vals.append(1.0 / self.dx)
            rows.append(2 * nt + k); cols.append(_vid1(nx, k, nx - 2)); vals.append(-1.0 / self.dx)
        return sp.csr_matrix((vals, (rows, cols)), shape=(self.m, self.n))

    def hess(self, u, lam):
        return sp.csr_matrix((self.n, self.n))

    def split(self, r):
        nt = self.nt
        return {"dirichlet": r[:nt], "mass": r[nt:2 * nt], "neumann": r[2 * nt:]}


FAMILIES = {MASS_IC: MassIC, FISHER_KPP: FisherKPP, BURGERS_LF: BurgersLF,
            DIFF2D_ENERGY: Diff2DEnergy, BURGERS_BC: BurgersBC, BURGERS_GODUNOV: BurgersGodunov}


def family_of(sample, **kw):
    """Build the oracle family object for one synthgen Sample."""
    f = sample.family
    if f == MASS_IC:
        return MassIC(sample.nx, sample.nt, sample.aux[: sample.nx], sample.aux[sample.nx], **kw)
    if f == FISHER_KPP:
        return FisherKPP(sample.nx, sample.nt, sample.aux[: sample.nx], sample.p0, sample.dt)
    if f == BURGERS_LF:
        return BurgersLF(sample.nx, sample.nt, sample.dt, sample.dx, sample.p0, sample.p1)
    if f == DIFF2D_ENERGY:
        return Diff2DEnergy(sample.nx, sample.ny, sample.nt, sample.dt, sample.dx,
                            sample.p0, sample.aux)
    if f == BURGERS_BC:
        return BurgersBC(sample.nx, sample.nt, sample.dx, sample.aux[0], sample.aux[1])
    if f == BURGERS_GODUNOV:
        return BurgersGodunov(sample.nx, sample.nt, sample.dt, sample.dx, sample.p0)
    raise ValueError(f"unknown family {f}")


def constraint_types(family: int):
    return FAMILIES[family].types


def real_fourier_basis(n):
    """Orthonormal real Fourier basis of R^n on the periodic grid x = 0..n-1
    (n even), as the columns of an n x n matrix, and the frequency of each
    column: 1/sqrt(n); sqrt(2/n) cos(2 pi k x/n), k = 1..n/2-1; (-1)^x/sqrt(n);
    sqrt(2/n) sin(2 pi k x/n), k = 1..n/2-1.  Every column is an eigenvector of
    the periodic second difference, with eigenvalue -4 sin^2(pi k/n)."""
    if n % 2:
        raise ValueError("the real Fourier basis here needs an even grid")
    x = np.arange(n)
    half = n // 2
    Q = np.empty((n, n))
    freq = np.empty(n, dtype=np.int64)
    Q[:, 0], freq[0] = 1.0 / np.sqrt(n), 0
    for k in range(1, half):
        Q[:, k], freq[k] = np.sqrt(2.0 / n) * np.cos(2 * np.pi * k * x / n), k
        Q[:, half + k], freq[half + k] = np.sqrt(2.0 / n) * np.sin(2 * np.pi * k * x / n), k
    Q[:, half], freq[half] = (-1.0) ** x / np.sqrt(n), half
    return Q, freq


class Diff2DEnergySpectral:
    """The 2D diffusion + per-frame energy family written in the orthonormal
    real Fourier basis of each frame: v_t = Q^T u_t Q (Q = real_fourier_basis,
    rows y, columns x), residual rows rotated by the same Q.  Because the
    periodic 5-point Laplacian is diagonal in that basis, the rows are

      residual rows  a(j,i) v_{k+1}(j,i) - v_k(j,i)      k = 0..Nt-2, modes (j, i)
      energy rows    sum_{j,i} v_t(j,i)^2 - E_t          t = 0..Nt-1

    with a(j,i) = 1 + dt*kappa*(4/dx^2)(sin^2(pi f_j/N) + sin^2(pi f_i/N)).
    The change of basis is orthogonal, so 1/2||u - u_hat||^2 = 1/2||v - v_hat||^2,
    the projection of v_hat is the transform of the projection of u_hat, and the
    residual multipliers transform back by the same Q (energy multipliers are
    unchanged)."""
    types = ("residual", "energy")

    def __init__(self, phys):
        if phys.nx != phys.ny:
            raise ValueError("square grids only")
        self.phys = phys
        self.nx = self.ny = phys.nx
        self.nt = phys.nt
        self.np_ = phys.np_
        self.n, self.m = phys.n, phys.m
        self.E = phys.E
        self.Q, f = real_fourier_basis(self.nx)
        s = np.sin(np.pi * f / self.nx) ** 2
        self.a = 1.0 + phys.dt * phys.kappa * (4.0 / (phys.dx * phys.dx)) * (s[:, None] + s[None, :])

    # orthogonal maps between the physical and spectral coordinates
    def to_spectral(self, u):
        U = np.asarray(u).reshape(-1, self.ny, self.nx)
        return np.einsum("yj,tyx,xi->tji", self.Q, U, self.Q).reshape(-1)

    def from_spectral(self, v):
        V = np.asarray(v).reshape(-1, self.ny, self.nx)
        return np.einsum("yj,tji,xi->tyx", self.Q, V, self.Q).reshape(-1)

    def lam_from_spectral(self, lam):
        k = (self.nt - 1) * self.np_
        return np.concatenate([self.from_spectral(lam[:k]), lam[k:]])

    def h(self, v):
        V = v.reshape(self.nt, self.np_)
        a = self.a.reshape(-1)
        res = a[None, :] * V[1:] - V[:-1]
        energy = (V * V).sum(axis=1) - self.E
        return np.concatenate([res.reshape(-1), energy])

    def jac(self, v):
        V = v.reshape(self.nt, self.np_)
        npt, nt = self.np_, self.nt
        a = self.a.reshape(-1)
        K, P = np.meshgrid(np.arange(nt - 1), np.arange(npt), indexing="ij")
        row = K * npt + P
        T, P2 = np.meshgrid(np.arange(nt), np.arange(npt), indexing="ij")
        rows = np.concatenate([row.ravel(), row.ravel(), ((nt - 1) * npt + T).ravel()])
        cols = np.concatenate([((K + 1) * npt + P).ravel(), (K * npt + P).ravel(), (T * npt + P2).ravel()])
        vals = np.concatenate([np.broadcast_to(a, K.shape).ravel(), -np.ones(K.size), 2.0 * V.ravel()])
        return sp.csr_matrix((vals, (rows, cols)), shape=(self.m, self.n))

    def hess(self, v, lam):
        lam_e = np.asarray(lam[(self.nt - 1) * self.np_:])
        return sp.diags(np.repeat(2.0 * lam_e, self.np_))

    def split(self, r):
        k = (self.nt - 1) * self.np_
        return {"residual": r[:k], "energy": r[k:]}
