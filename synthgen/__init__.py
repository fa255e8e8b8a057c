"""Seeded synthetic inputs for the batched constraint projection.

This module only draws random fields and packs them; it holds none of the
projection's arithmetic.  Both the CPU oracle and the GPU library consume what
it produces.  The trained flow-matching models and PDE datasets the paper
samples from are not available, so seeded fields with the shapes and value
ranges of the paper's 1D/2D workloads stand in for the intermediate states
u_hat that the projection receives (paper Sec. II-A, eqs. for the forward
shoot and the projection; problem shapes in Appendix A).

Families (the integer codes match the C header):
  1  MASS_IC     initial condition + per-step mass (Appendix A, heat problem;
                 Appendix C encoding of the mass rows)
  2  FISHER_KPP  initial condition + nonlinear mass budget of a logistic
                 reaction (Appendix A reaction-diffusion; Appendix D
                 discretization of the conservation law)
  3  BURGERS_LF  local flux-update residuals of viscous Burgers with the
                 smooth Lax-Friedrichs flux (Appendix D flux residual)
  4  DIFF2D_ENERGY  implicit 2D diffusion residuals + per-frame quadratic
                 invariant (Appendix A Navier-Stokes analogue)
  5  BURGERS_BC  Dirichlet row on the left boundary, mass row and Neumann row
                 on the right boundary per time step (Appendix A, the first
                 Burgers regime; Appendix D discretizations)
  6  BURGERS_GODUNOV  local flux-update residuals of Burgers with Godunov's
                 flux (Appendix D, Godunov's flux conservation), periodic

Every field is float64.  Layout of one sample: time slab major, then y, then x
(x fastest), which is the paper's flattening of the space-time grid
(Appendix C).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

F1_MASS_IC = 1
F2_FISHER_KPP = 2
F3_BURGERS_LF = 3
F4_DIFF2D_ENERGY = 4
F5_BURGERS_BC = 5
F6_BURGERS_GODUNOV = 6

FAMILY_NAMES = {1: "mass_ic", 2: "fisher_kpp", 3: "burgers_lf", 4: "diff2d_energy", 5: "burgers_bc",
                6: "burgers_godunov"}


def n_rows(family: int, nx: int, ny: int, nt: int) -> int:
    """Number of constraint rows of one sample, canonical encoding."""
    if family in (F1_MASS_IC, F2_FISHER_KPP):
        return nx + nt - 1
    if family in (F3_BURGERS_LF, F6_BURGERS_GODUNOV):
        return nx * (nt - 1)
    if family == F4_DIFF2D_ENERGY:
        return (nt - 1) * nx * ny + nt
    if family == F5_BURGERS_BC:
        return 3 * nt
    raise ValueError(f"unknown family {family}")


def n_aux(family: int, nx: int, ny: int, nt: int) -> int:
    if family == F1_MASS_IC:
        return nx + 1          # g[nx], M0
    if family == F2_FISHER_KPP:
        return nx              # g[nx]
    if family in (F3_BURGERS_LF, F6_BURGERS_GODUNOV):
        return 0
    if family == F4_DIFF2D_ENERGY:
        return nt              # E[nt]
    if family == F5_BURGERS_BC:
        return 2               # u_L, m0
    raise ValueError(f"unknown family {family}")


@dataclass
class Sample:
    family: int
    nx: int
    ny: int
    nt: int
    dt: float
    dx: float
    p0: float = 0.0
    p1: float = 0.0
    uhat: np.ndarray = None     # shape (nt, ny, nx) or (nt, nx)
    aux: np.ndarray = None      # 1-D, length n_aux

    @property
    def n(self) -> int:
        return self.nx * self.ny * self.nt

    @property
    def m(self) -> int:
        return n_rows(self.family, self.nx, self.ny, self.nt)


@dataclass
class Batch:
    samples: List[Sample]
    name: str = ""
    # packed views, filled by pack()
    uhat: Optional[np.ndarray] = None
    aux: Optional[np.ndarray] = None
    var_off: Optional[np.ndarray] = None
    row_off: Optional[np.ndarray] = None
    aux_off: Optional[np.ndarray] = None
    meta: dict = field(default_factory=dict)

    def __len__(self):
        return len(self.samples)

    @property
    def total_vars(self) -> int:
        return int(sum(s.n for s in self.samples))

    @property
    def total_rows(self) -> int:
        return int(sum(s.m for s in self.samples))

    @property
    def uniform(self) -> bool:
        s0 = self.samples[0]
        return all((s.family, s.nx, s.ny, s.nt) == (s0.family, s0.nx, s0.ny, s0.nt)
                   for s in self.samples)

    def pack(self) -> "Batch":
        nv = np.array([s.n for s in self.samples], dtype=np.int64)
        nr = np.array([s.m for s in self.samples], dtype=np.int64)
        na = np.array([len(s.aux) for s in self.samples], dtype=np.int64)
        self.var_off = np.concatenate([[0], np.cumsum(nv)[:-1]]).astype(np.int64)
        self.row_off = np.concatenate([[0], np.cumsum(nr)[:-1]]).astype(np.int64)
        self.aux_off = np.concatenate([[0], np.cumsum(na)[:-1]]).astype(np.int64)
        self.uhat = np.concatenate([s.uhat.reshape(-1) for s in self.samples]).astype(np.float64)
        if na.sum() > 0:
            self.aux = np.concatenate([s.aux.reshape(-1) for s in self.samples]).astype(np.float64)
        else:
            self.aux = np.zeros(1, dtype=np.float64)
        return self

    def unpack_vars(self, flat: np.ndarray) -> List[np.ndarray]:
        out = []
        for s, off in zip(self.samples, self.var_off):
            out.append(np.asarray(flat[off:off + s.n]).reshape(s.uhat.shape))
        return out

    def unpack_rows(self, flat: np.ndarray) -> List[np.ndarray]:
        return [np.asarray(flat[off:off + s.m]) for s, off in zip(self.samples, self.row_off)]


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


# --------------------------------------------------------------------------
# per-family recipes (one sample each, drawing from the shared generator)
# --------------------------------------------------------------------------

def _draw_f1(rng, nx, nt, noise=0.1) -> Sample:
    # cell centres and half-wave sine modes, so the mass of g is generically nonzero
    x = (np.arange(nx) + 0.5) / nx
    modes = np.stack([np.sin(k * np.pi * x) for k in range(1, 5)])      # (4, nx)
    b = rng.standard_normal(4)
    a = rng.standard_normal(4)
    g = b @ modes
    m0 = float(g.sum())
    base = a @ modes
    uhat = np.broadcast_to(base, (nt, nx)) + noise * rng.standard_normal((nt, nx))
    aux = np.concatenate([g, [m0]])
    return Sample(F1_MASS_IC, nx, 1, nt, dt=1.0 / max(nt - 1, 1), dx=1.0 / nx,
                  uhat=np.ascontiguousarray(uhat), aux=aux)


def _draw_f2(rng, nx, nt, dt=0.01, noise=0.05) -> Sample:
    x = np.arange(nx) / nx
    rho = rng.uniform(0.5, 2.0)
    z = np.zeros(nx)
    for _ in range(3):
        amp = rng.normal(0.0, 2.0)
        c = rng.uniform(0.0, 1.0)
        w = rng.uniform(0.05, 0.15)
        d = np.abs(x - c)
        d = np.minimum(d, 1.0 - d)              # periodic distance on [0, 1)
        z += amp * np.exp(-d * d / (2.0 * w * w))
    g = 1.0 / (1.0 + np.exp(-z))
    uhat = np.broadcast_to(g, (nt, nx)) + noise * rng.standard_normal((nt, nx))
    return Sample(F2_FISHER_KPP, nx, 1, nt, dt=dt, dx=1.0 / nx, p0=rho,
                  uhat=np.ascontiguousarray(uhat), aux=g.copy())


def _lf_burgers_update(u, dt, dx, nu, alpha):
    """One explicit conservative update of viscous Burgers with the smooth
    Lax-Friedrichs interface flux, periodic in x (input synthesis only)."""
    up = np.roll(u, -1)
    flux_half = 0.25 * (u * u + up * up) - 0.5 * alpha * (up - u)     # F_{i+1/2}
    flux_diff = flux_half - np.roll(flux_half, 1)                      # F_{i+1/2} - F_{i-1/2}
    visc = nu * (up - 2.0 * u + np.roll(u, 1)) / (dx * dx)
    return u - (dt / dx) * flux_diff + dt * visc


def _draw_f3(rng, nx, nt, dt=1e-3, nu=0.01, alpha=1.0, noise=0.02) -> Sample:
    x = np.arange(nx) / nx
    u0 = np.zeros(nx)
    for k in range(1, 5):
        a, b = rng.standard_normal(2)
        u0 += (a * np.cos(2 * np.pi * k * x) + b * np.sin(2 * np.pi * k * x)) / k
    u0 *= 0.8 / max(np.abs(u0).max(), 1e-12)
    dx = 1.0 / nx
    traj = np.empty((nt, nx))
    traj[0] = u0
    xi = noise * rng.standard_normal((nt - 1, nx))
    for k in range(nt - 1):
        traj[k + 1] = _lf_burgers_update(traj[k], dt, dx, nu, alpha) + xi[k]
    return Sample(F3_BURGERS_LF, nx, 1, nt, dt=dt, dx=dx, p0=nu, p1=alpha,
                  uhat=traj, aux=np.zeros(0))


def _godunov_bc_trajectory(u0, nt, dt, dx, u_left):
    """Inviscid Burgers by Godunov's finite-volume method with the left
    boundary held at u_left and a zero-gradient right boundary, saved every dt
    (CFL-limited substeps); input synthesis only."""
    def flux(a, b):
        # Godunov flux of f(u) = u^2 / 2 between states a (left) and b (right)
        return np.maximum(0.5 * np.maximum(a, 0.0) ** 2, 0.5 * np.minimum(b, 0.0) ** 2)
    traj = np.empty((nt, u0.size))
    u = u0.copy()
    u[0] = u_left
    traj[0] = u
    for k in range(1, nt):
        t = 0.0
        while t < dt - 1e-15:
            h = min(dt - t, 0.45 * dx / max(np.abs(u).max(), 1e-12))
            ghost = np.concatenate([[u_left], u, [u[-1]]])
            f = flux(ghost[:-1], ghost[1:])            # interfaces i-1/2, i = 0..nx
            u = u - (h / dx) * (f[1:] - f[:-1])
            u[0] = u_left
            t += h
        traj[k] = u
    return traj


def _draw_f5(rng, nx, nt, noise=0.05) -> Sample:
    # the paper's Burgers-BC setting: front 1 / (1 + exp((x - p) / eps)),
    # eps = 0.02, p ~ U(0.2, 0.8); left boundary value u_bc ~ U(0, 1); grid
    # with both ends on [0, 1] and t in [0, 1]
    dx = 1.0 / (nx - 1)
    dt = 1.0 / max(nt - 1, 1)
    x = np.arange(nx) * dx
    p = rng.uniform(0.2, 0.8)
    u_left = rng.uniform(0.0, 1.0)
    u0 = 1.0 / (1.0 + np.exp((x - p) / 0.02))
    m0 = float(dx * u0.sum())
    clean = _godunov_bc_trajectory(u0, nt, dt, dx, u_left)
    uhat = clean + noise * rng.standard_normal(clean.shape)
    return Sample(F5_BURGERS_BC, nx, 1, nt, dt=dt, dx=dx, uhat=uhat,
                  aux=np.array([u_left, m0]))


def _godunov_periodic_update(u, dt, dx, nu):
    """One explicit step of Burgers with Godunov's interface flux and a
    centred viscous term, periodic in x (input synthesis only)."""
    up = np.roll(u, -1)
    a, b = np.maximum(u, 0.0), np.minimum(up, 0.0)
    flux_half = np.maximum(0.5 * a * a, 0.5 * b * b)                   # F_{i+1/2}
    visc = nu * (up - 2.0 * u + np.roll(u, 1)) / (dx * dx)
    return u - (dt / dx) * (flux_half - np.roll(flux_half, 1)) + dt * visc


def _draw_f6(rng, nx, nt, dt=1e-3, nu=0.0, noise=0.02) -> Sample:
    # random four-mode Fourier initial condition (it changes sign, so the
    # trajectory holds shocks, expansions and the flux's kinks), scaled to
    # max |u| = 0.8, explicit Godunov steps plus N(0, noise^2) per step
    x = np.arange(nx) / nx
    u0 = np.zeros(nx)
    for k in range(1, 5):
        a, b = rng.standard_normal(2)
        u0 += (a * np.cos(2 * np.pi * k * x) + b * np.sin(2 * np.pi * k * x)) / k
    u0 *= 0.8 / max(np.abs(u0).max(), 1e-12)
    dx = 1.0 / nx
    traj = np.empty((nt, nx))
    traj[0] = u0
    xi = noise * rng.standard_normal((nt - 1, nx))
    for k in range(nt - 1):
        traj[k + 1] = _godunov_periodic_update(traj[k], dt, dx, nu) + xi[k]
    return Sample(F6_BURGERS_GODUNOV, nx, 1, nt, dt=dt, dx=dx, p0=nu,
                  uhat=traj, aux=np.zeros(0))


def _draw_f4(rng, n, nt, dt=0.01, noise=0.05) -> Sample:
    kappa = rng.uniform(0.01, 0.1)
    h = 1.0 / n
    kx = np.fft.fftfreq(n, d=1.0 / n)
    KX, KY = np.meshgrid(kx, kx, indexing="xy")      # KX varies along x (last axis)
    kmag = np.sqrt(KX ** 2 + KY ** 2)
    amp = np.zeros_like(kmag)
    nz = kmag > 0
    amp[nz] = kmag[nz] ** (-1.5)                      # energy spectrum ~ k^-3
    coef = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) * amp
    u0 = np.real(np.fft.ifft2(coef))
    u0 -= u0.mean()
    u0 /= u0.std()
    # exact implicit-Euler heat steps on the periodic grid, done spectrally
    sym = (np.sin(np.pi * KX / n) ** 2 + np.sin(np.pi * KY / n) ** 2) * (4.0 / (h * h))
    decay = 1.0 / (1.0 + dt * kappa * sym)
    clean = np.empty((nt, n, n))
    clean[0] = u0
    uk = np.fft.fft2(u0)
    for k in range(1, nt):
        uk = uk * decay
        clean[k] = np.real(np.fft.ifft2(uk))
    energy = (clean ** 2).reshape(nt, -1).sum(axis=1)
    uhat = clean + noise * rng.standard_normal(clean.shape)
    return Sample(F4_DIFF2D_ENERGY, n, n, nt, dt=dt, dx=h, p0=kappa,
                  uhat=uhat, aux=energy)


# --------------------------------------------------------------------------
# batches
# --------------------------------------------------------------------------

def mass_ic_batch(batch=32, nx=64, nt=32, seed=1001) -> Batch:
    rng = _rng(seed)
    return Batch([_draw_f1(rng, nx, nt) for _ in range(batch)], name="mass_ic").pack()


def fisher_kpp_batch(batch=256, nx=128, nt=100, dt=0.01, seed=2001) -> Batch:
    rng = _rng(seed)
    return Batch([_draw_f2(rng, nx, nt, dt) for _ in range(batch)], name="fisher_kpp").pack()


def burgers_batch(batch=512, nx=128, nt=128, dt=1e-3, nu=0.01, alpha=1.0, seed=3001) -> Batch:
    rng = _rng(seed)
    return Batch([_draw_f3(rng, nx, nt, dt, nu, alpha) for _ in range(batch)],
                 name="burgers_lf").pack()


def burgers_bc_batch(batch=512, nx=101, nt=101, seed=6001) -> Batch:
    rng = _rng(seed)
    return Batch([_draw_f5(rng, nx, nt) for _ in range(batch)], name="burgers_bc").pack()


def godunov_batch(batch=512, nx=101, nt=11, dt=0.005, nu=0.0, seed=7001) -> Batch:
    rng = _rng(seed)
    return Batch([_draw_f6(rng, nx, nt, dt=dt, nu=nu) for _ in range(batch)], name="burgers_godunov").pack()


def diff2d_batch(batch=128, n=64, nt=16, dt=0.01, seed=4001) -> Batch:
    rng = _rng(seed)
    return Batch([_draw_f4(rng, n, nt, dt) for _ in range(batch)], name="diff2d_energy").pack()


RAGGED_NX = (64, 96, 128, 192, 256)
RAGGED_NT = (32, 64, 128)


def ragged_batch(batch=1024, seed=5001, nx_choices=RAGGED_NX, nt_choices=RAGGED_NT,
                 families=(F1_MASS_IC, F2_FISHER_KPP, F3_BURGERS_LF)) -> Batch:
    """Mixed families and grid sizes.  Burgers time steps shrink with Nx^2 so the
    explicit generator stays monotone (dt = 1e-3 * min(1, (128/Nx)^2))."""
    rng = _rng(seed)
    out = []
    for _ in range(batch):
        fam = int(families[rng.integers(len(families))])
        nx = int(nx_choices[rng.integers(len(nx_choices))])
        nt = int(nt_choices[rng.integers(len(nt_choices))])
        if fam == F1_MASS_IC:
            out.append(_draw_f1(rng, nx, nt))
        elif fam == F2_FISHER_KPP:
            out.append(_draw_f2(rng, nx, nt))
        else:
            dt = 1e-3 * min(1.0, (128.0 / nx) ** 2)
            out.append(_draw_f3(rng, nx, nt, dt=dt))
    return Batch(out, name="ragged").pack()


def upstream_grad(b: Batch, seed: int = 7) -> np.ndarray:
    """N(0,1) upstream gradient dL/du, packed like the variables."""
    return _rng(seed).standard_normal(b.total_vars)


def prior_sample(b: Batch, seed: int = 11) -> np.ndarray:
    """N(0,1) draw from the flow's source distribution, packed like the variables."""
    return _rng(seed).standard_normal(b.total_vars)


# the five benchmark configurations, by name, at full size
CONFIGS = {
    "mass_ic": dict(fn=mass_ic_batch, kw=dict(batch=32, nx=64, nt=32, seed=1001)),
    "fisher_kpp": dict(fn=fisher_kpp_batch, kw=dict(batch=256, nx=128, nt=100, seed=2001)),
    "burgers_lf": dict(fn=burgers_batch, kw=dict(batch=512, nx=128, nt=128, seed=3001)),
    # 6 frames: the energy rows of one diffusion trajectory are nearly
    # dependent, the more so the more frames (condition number of their
    # reduced Jacobian about 5e3 at 64 x 64 x 6, 3e5 at x 8, 5e11 at x 16,
    # where float64 no longer determines the projection)
    "diff2d_energy": dict(fn=diff2d_batch, kw=dict(batch=128, n=64, nt=6, seed=4001)),
    "ragged": dict(fn=ragged_batch, kw=dict(batch=1024, seed=5001)),
    # the paper's first Burgers regime (boundary rows + mass) on its 101 x 101 grid
    "burgers_bc": dict(fn=burgers_bc_batch, kw=dict(batch=512, nx=101, nt=101, seed=6001)),
    # the flux-residual rows of the paper's Godunov regime with ten flux steps
    # (its Flux(10) case) on the paper's 101-point grid
    "burgers_godunov": dict(fn=godunov_batch, kw=dict(batch=512, nx=101, nt=11, dt=0.005, seed=7001)),
}


def make(name: str, **override) -> Batch:
    spec = CONFIGS[name]
    kw = dict(spec["kw"])
    kw.update(override)
    return spec["fn"](**kw)
