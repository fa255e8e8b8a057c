"""Constrained flow-matching sampling loop around the projection (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The sampler of Sec. II-A discretizes flow time [0, 1] into N uniform
substeps.  At flow time tau (next tau' = tau + 1/N) it
  1. shoots to flow time 1 with the velocity: u1_hat = u_tau + (1 - tau) v(u_tau, tau),
  2. projects: u1 = argmin 1/2 ||u - u1_hat||^2  s.t.  h(u) = 0,
  3. pulls back along the straight-line interpolant: u_tau' = u0 + tau' (u1 - u0),
and the sample is the projection of the last substep (tau' = 1).  The
penalized correction the paper mentions and omits is omitted here too.

The trained velocity network is not available; the velocity used is the
exact one of a Gaussian target: for the straight-line interpolant
x_tau = (1 - tau) x0 + tau x1 between independent x0 ~ N(0, I) and
x1 ~ N(m, s^2 I), the marginal velocity E[x1 - x0 | x_tau = u] is affine,

    v(u, tau) = m + c(tau) (u - tau m),
    c(tau) = (tau s^2 - (1 - tau)) / ((1 - tau)^2 + tau^2 s^2)

(the conditional expectation of one jointly Gaussian vector given another).
Pins (tests/test_oracle_pcfm.py): Monte-Carlo regression of x1 - x0 on
x_tau, the special values c(0) = -1 (the first shoot lands on the target
mean) and c(1) = 1, and feasibility of the sample.
"""
from __future__ import annotations

import numpy as np

from .kkt import project_sample


def gaussian_ot_velocity(u, tau, mean, s):
    """E[x1 - x0 | x_tau = u] for x0 ~ N(0, I), x1 ~ N(mean, s^2 I)."""
    var = (1.0 - tau) ** 2 + tau * tau * s * s
    c = (tau * s * s - (1.0 - tau)) / var
    return mean + c * (u - tau * mean)


def pcfm_sample(fam, u0, mean, s, nsteps, return_history=False):
    """Run the N-substep sampler for one sample.  Returns the sample (and
    optionally the list of projected candidates u1 of every substep)."""
    u0 = np.asarray(u0, dtype=np.float64).reshape(-1)
    mean = np.asarray(mean, dtype=np.float64).reshape(-1)
    u = u0.copy()
    hist = []
    u1 = u0
    for j in range(nsteps):
        tau, tau_next = j / nsteps, (j + 1) / nsteps
        u1_hat = u + (1.0 - tau) * gaussian_ot_velocity(u, tau, mean, s)
        u1, _ = project_sample(fam, u1_hat)
        hist.append(u1)
        u = u0 + tau_next * (u1 - u0)
    return (u1, hist) if return_history else u1
