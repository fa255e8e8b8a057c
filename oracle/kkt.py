"""Newton-KKT projection and its implicit-function adjoint (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Forward (paper Appendix B, the Newton-KKT system; projection problem of
Sec. II-A / III-B).  With f(u) = 1/2 ||u - u_hat||^2 and the Lagrangian
L(u, lam) = f(u) + lam^T h(u) (the printed Lagrangian in Appendix B writes
J^T lam where lam^T h is meant; the KKT conditions printed just above it are
the ones used), one Newton-Raphson step on

    F(u, lam) = [ u - u_hat + J(u)^T lam ; h(u) ] = 0

solves  [[W, J^T], [J, 0]] [du; dlam] = -F,   W = I + sum_i lam_i Hess h_i,

here with a general sparse LU (scipy SuperLU) on the full (n+m)x(n+m)
matrix.  Start (u, lam) = (u_hat, 0).  Steps are damped by halving until the
2-norm of F decreases (the textbook safeguard of Newton-Raphson for F = 0;
near the solution the full step is always taken); iterate until ||F||_inf
stops shrinking (round-off floor) or falls below `atol`.  The result is the KKT
point; for linear h it is the affine projection
u_hat - A^T (A A^T)^{-1} (A u_hat - b) (paper Table 1 row 'Au - b').

Adjoint.  Differentiating F(u*, lam*; u_hat) = 0 gives
K [du; dlam] = [du_hat; 0] with the symmetric K = [[W, J^T], [J, 0]] at the
solution, so the vector-Jacobian product of u* with respect to u_hat is the
u-block of K^{-1} [g; 0].

Parity: pinned by closed forms (affine projection with A probed from h,
sphere projection), finite-difference Jacobians in the KKT check, an
independent SQP solver on tiny grids, and central differences of the forward
for the adjoint (tests/test_oracle_pins.py, tests/test_oracle_adjoint.py).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .families import family_of


def _kkt_matrix(fam, u, lam):
    J = fam.jac(u)
    W = sp.identity(fam.n, format="csr") + fam.hess(u, lam)
    K = sp.bmat([[W, J.T], [J, None]], format="csc")
    return K, J


def kkt_residual(fam, u, uhat, lam):
    """(stationarity u - u_hat + J^T lam, feasibility h(u))"""
    J = fam.jac(u)
    return u - uhat + J.T @ lam, fam.h(u)


def project_sample(fam, uhat, max_iter=100, atol=0.0, return_info=False):
    """Project one flattened sample onto {h = 0}.  Returns (u, lam[, info])."""
    uhat = np.asarray(uhat, dtype=np.float64).reshape(-1)
    n, m = fam.n, fam.m
    u = uhat.copy()
    lam = np.zeros(m)
    if m == 0:
        info = dict(iters=0, res=0.0, history=[])
        return (u, lam, info) if return_info else (u, lam)
    best = None
    history = []
    stall = 0
    for it in range(max_iter):
        K, J = _kkt_matrix(fam, u, lam)
        ru = u - uhat + J.T @ lam
        rh = fam.h(u)
        res = max(np.abs(ru).max(initial=0.0), np.abs(rh).max(initial=0.0))
        res2 = np.sqrt(np.dot(ru, ru) + np.dot(rh, rh))
        history.append(res)
        # progress is judged on the 2-norm, which the damped step decreases
        if best is None or res2 < best[0]:
            best = (res2, u.copy(), lam.copy(), it, res)
            stall = 0
        else:
            stall += 1
        if res <= atol or stall >= 2:
            break
        step = spla.spsolve(K, -np.concatenate([ru, rh]))
        # damped Newton-Raphson: halve the step until the 2-norm of the KKT
        # residual F decreases (full steps near the solution)
        f0 = np.sqrt(np.dot(ru, ru) + np.dot(rh, rh))
        alpha = 1.0
        for _ in range(40):
            ut, lt = u + alpha * step[:n], lam + alpha * step[n:]
            rut, rht = kkt_residual(fam, ut, uhat, lt)
            if np.sqrt(np.dot(rut, rut) + np.dot(rht, rht)) <= (1.0 - 1e-4 * alpha) * f0 or f0 < 1e-12:
                break
            alpha *= 0.5
        u, lam = ut, lt
    _, u, lam, it, res = best
    info = dict(iters=it, res=res, history=history)
    return (u, lam, info) if return_info else (u, lam)


def adjoint_sample(fam, u, lam, grad_u):
    """d(u*)/d(u_hat)^T grad_u at the KKT point (u, lam)."""
    n, m = fam.n, fam.m
    g = np.asarray(grad_u, dtype=np.float64).reshape(-1)
    if m == 0:
        return g.copy()
    K, _ = _kkt_matrix(fam, u, lam)
    sol = spla.spsolve(K, np.concatenate([g, np.zeros(m)]))
    return sol[:n]


def project_batch(batch, max_iter=100, indices=None):
    """Project every sample of a synthgen Batch.  Returns packed (u, lam, iters)."""
    idx = range(len(batch)) if indices is None else indices
    u_out = np.array(batch.uhat, copy=True)
    lam_out = np.zeros(batch.total_rows)
    iters = np.zeros(len(batch), dtype=np.int32)
    for s in idx:
        smp = batch.samples[s]
        fam = family_of(smp)
        u, lam, info = project_sample(fam, smp.uhat.reshape(-1), max_iter=max_iter, return_info=True)
        vo, ro = batch.var_off[s], batch.row_off[s]
        u_out[vo:vo + smp.n] = u
        lam_out[ro:ro + smp.m] = lam
        iters[s] = info["iters"]
    return u_out, lam_out, iters


def adjoint_batch(batch, u_packed, lam_packed, grad_packed, indices=None):
    idx = range(len(batch)) if indices is None else indices
    out = np.zeros(batch.total_vars)
    for s in idx:
        smp = batch.samples[s]
        fam = family_of(smp)
        vo, ro = batch.var_off[s], batch.row_off[s]
        out[vo:vo + smp.n] = adjoint_sample(fam, u_packed[vo:vo + smp.n],
                                            lam_packed[ro:ro + smp.m],
                                            grad_packed[vo:vo + smp.n])
    return out
