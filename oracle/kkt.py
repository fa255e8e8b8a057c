"""Newton/SQP projection with an l1-merit line search, and its adjoint (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Forward (projection step of Sec. II-A, restated as an NLP in Sec. III-B; the
Newton-KKT system of Appendix B).  With f(u) = 1/2 ||u - u_hat||^2 and the
Lagrangian L(u, lam) = f(u) + lam^T h(u) (the printed Lagrangian in
Appendix B writes J^T lam where lam^T h is meant; the KKT conditions printed
just above it are the ones used), every iteration solves the full Newton-KKT
system

    [[W, J^T], [J, 0]] [p; lam_plus] = -[u - u_hat; h(u)]

for the primal step p and the new multipliers lam_plus, with a general sparse
LU (scipy SuperLU) on the whole (n+m)x(n+m) matrix: no Schur reduction, no
ordering, no band structure.  W is the Lagrangian Hessian I + sum_i lam_i
Hess h_i, which is diagonal for every family here.  The iteration is the
textbook SQP method for equality constraints with the l1 merit function
(Nocedal & Wright, Numerical Optimization, ch. 18, Algorithm 18.3):

  * away from the solution W is the exact Hessian with its entries raised to
    at least W_FLOOR, so the step is a descent direction of the merit;
  * once ||h||_inf <= LOCAL_H the exact Hessian is used, as long as the step
    it gives is still a descent direction (then Newton's local quadratic
    convergence takes over);
  * merit phi(u) = 1/2 ||u - u_hat||^2 + mu ||h(u)||_1 with
    mu = max(mu, 1.1 ||lam_plus||_inf + 1e-8); the change of phi along the
    step is computed as the exact algebraic difference
    a (u - u_hat).p + a^2/2 ||p||^2 + mu (||h(u + a p)||_1 - ||h(u)||_1),
    never as a difference of two phi values;
  * Armijo test phi(u + a p) - phi(u) <= 1e-4 a D with the directional
    derivative D = (u - u_hat).p - mu ||h(u)||_1; a is halved up to 30 times;
    if a = 1 fails, one second-order correction q (the same KKT matrix with
    right-hand side [0; -h(u + p)]) is tried on u + p + q first;
  * multipliers move with the step: lam <- lam + a (lam_plus - lam).

It starts from (u_hat, 0) and runs to stagnation: until the KKT residual
max(||u - u_hat + J^T lam||_inf, ||h||_inf) stops decreasing for two
iterations in the local phase, or the step falls below round-off.  The point
with the smallest KKT residual seen in the local phase is returned, and it is
checked: unless its feasibility and stationarity are below CONV_TOL (relative
to 1 + ||u_hat||_inf for stationarity), project_sample raises
OracleNotConverged.  For linear h the result is the affine projection
u_hat - A^T (A A^T)^{-1} (A u_hat - b) (paper Table 1 row 'Au - b').

Adjoint.  Differentiating F(u*, lam*; u_hat) = [u - u_hat + J^T lam; h] = 0
gives K [du; dlam] = [du_hat; 0] with the symmetric K = [[W, J^T], [J, 0]] at
the solution (exact W), so the vector-Jacobian product of u* with respect to
u_hat is the u-block of K^{-1} [g; 0].

Parity: pinned by closed forms (affine projection with A probed from h,
sphere projection), finite-difference Jacobians in the KKT check,
second-order sufficiency on null(J), an independent SQP solver (SLSQP) on
tiny grids, and central differences of the forward for the adjoint
(tests/test_oracle_pins.py, tests/test_oracle_adjoint.py,
tests/test_oracle_globalization.py).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .families import Diff2DEnergySpectral, family_of

W_FLOOR = 0.1       # smallest Hessian entry used by a globalized step
LOCAL_H = 1e-6      # ||h||_inf below which exact-Hessian steps are tried
ARMIJO = 1e-4
MAX_HALVINGS = 30
CONV_TOL = 1e-10    # acceptance of the returned point


class OracleNotConverged(RuntimeError):
    """The oracle's SQP iteration did not reach a KKT point within CONV_TOL."""


def _hess_diag(fam, u, lam):
    H = sp.csr_matrix(fam.hess(u, lam))
    d = H.diagonal()
    off = H - sp.diags(d)
    if off.count_nonzero():
        raise ValueError("the oracle's SQP step needs a diagonal Lagrangian Hessian")
    return 1.0 + d


def _kkt_lu(J, w):
    K = sp.bmat([[sp.diags(w), J.T], [J, None]], format="csc")
    return spla.splu(K)


def kkt_residual(fam, u, uhat, lam):
    """(stationarity u - u_hat + J^T lam, feasibility h(u))"""
    J = fam.jac(u)
    return u - uhat + J.T @ lam, fam.h(u)


def _kkt_inf(fam, u, uhat, lam):
    ru, rh = kkt_residual(fam, u, uhat, lam)
    return float(np.abs(ru).max(initial=0.0)), float(np.abs(rh).max(initial=0.0))


def _spectral_form(fam, basis):
    if basis == "physical":
        return None
    if basis != "spectral":
        raise ValueError(basis)
    if getattr(fam, "types", None) == ("residual", "energy") and not hasattr(fam, "phys") \
            and fam.nx == fam.ny and fam.nx % 2 == 0:
        return Diff2DEnergySpectral(fam)
    return None


def project_sample(fam, uhat, max_iter=200, return_info=False, strict=True, basis="spectral"):
    """Project one flattened sample onto {h = 0}.  Returns (u, lam[, info]).

    info: iters, converged, h_inf, stat_inf (at the returned point),
    objective 1/2||u - u_hat||^2, backtracks, soc (accepted corrections),
    clamped (iterations whose step used a shifted Hessian), history.

    The 2D diffusion + energy family is solved in the orthonormal real Fourier
    basis of each frame (basis="spectral", the default for it): the same
    problem in rotated coordinates, whose Newton-KKT matrix has one small
    block per Fourier mode plus the energy rows, so the sparse LU stays
    cheap; u and the residual multipliers are rotated back.  The reported
    h_inf and stat_inf are then those of the physical rows.
    basis="physical" solves every family in its own variables."""
    sf = _spectral_form(fam, basis)
    if sf is not None:
        v, lv, info = project_sample(sf, sf.to_spectral(uhat), max_iter=max_iter,
                                     return_info=True, strict=False, basis="physical")
        u, lam = sf.from_spectral(v), sf.lam_from_spectral(lv)
        uh = np.asarray(uhat, dtype=np.float64).reshape(-1)
        s_inf, h_inf = _kkt_inf(fam, u, uh, lam)
        scale = 1.0 + float(np.abs(uh).max(initial=0.0))
        info.update(h_inf=h_inf, stat_inf=s_inf,
                    converged=h_inf <= CONV_TOL and s_inf <= CONV_TOL * scale)
        if strict and not info["converged"]:
            raise OracleNotConverged(
                f"oracle SQP stopped at ||h||_inf = {h_inf:.3e}, stationarity {s_inf:.3e}")
        return (u, lam, info) if return_info else (u, lam)
    uhat = np.asarray(uhat, dtype=np.float64).reshape(-1)
    n, m = fam.n, fam.m
    u = uhat.copy()
    lam = np.zeros(m)
    scale = 1.0 + float(np.abs(uhat).max(initial=0.0))
    if m == 0:
        info = dict(iters=0, converged=True, h_inf=0.0, stat_inf=0.0, objective=0.0,
                    backtracks=0, soc=0, clamped=0, history=[])
        return (u, lam, info) if return_info else (u, lam)
    mu = 0.0
    best = None
    stall = 0
    history = []
    backtracks = soc_taken = clamped = 0
    it = 0
    for it in range(max_iter + 1):
        h = fam.h(u)
        J = fam.jac(u)
        ru = u - uhat + J.T @ lam
        s_inf = float(np.abs(ru).max(initial=0.0))
        h_inf = float(np.abs(h).max(initial=0.0))
        res = max(h_inf, s_inf / scale)
        history.append(res)
        if h_inf <= LOCAL_H:
            if best is None or res < best[0]:
                best = (res, u.copy(), lam.copy(), it, h_inf, s_inf)
                stall = 0
            else:
                stall += 1
            if res == 0.0 or stall >= 2:
                break
        if it == max_iter:
            break
        d = u - uhat
        w_exact = _hess_diag(fam, u, lam)
        h1 = float(np.abs(h).sum())

        def step_with(w):
            lu = _kkt_lu(J, w)
            sol = lu.solve(-np.concatenate([d, h]))
            return lu, sol[:n], sol[n:]

        def merit_dir(w):
            lu, p, lam_plus = step_with(w)
            mu_t = max(mu, 1.1 * float(np.abs(lam_plus).max(initial=0.0)) + 1e-8)
            return lu, p, lam_plus, mu_t, float(d @ p) - mu_t * h1

        def dphi(p, mu_t, alpha, ut):
            return (alpha * float(d @ p) + 0.5 * alpha * alpha * float(p @ p)
                    + mu_t * (float(np.abs(fam.h(ut)).sum()) - h1))

        def full_or_soc(lu, p, mu_t, D):
            ut = u + p
            if dphi(p, mu_t, 1.0, ut) <= ARMIJO * D:
                return ut, 0
            q = lu.solve(np.concatenate([np.zeros(n), -fam.h(ut)]))[:n]
            uq = ut + q
            if dphi(uq - u, mu_t, 1.0, uq) <= ARMIJO * D:
                return uq, 1
            return None, 0

        accepted = False
        alpha = 1.0
        # 1) the Newton step with the exact Lagrangian Hessian, taken whole
        #    (or with one second-order correction) when it passes the test
        lu, p, lam_plus, mu_t, D = merit_dir(w_exact)
        tiny = np.abs(p).max(initial=0.0) <= 1e-15 * scale
        if tiny and h_inf <= LOCAL_H:
            # the Newton step is below round-off: only the multipliers move
            lam = lam_plus
            continue
        if D < 0.0:
            ut, s = full_or_soc(lu, p, mu_t, D)
            if ut is not None:
                accepted, soc_taken, mu = True, soc_taken + s, mu_t
        # 2) otherwise the step with W raised to at least W_FLOOR (a descent
        #    direction of the merit), backtracked
        if not accepted:
            w = np.maximum(w_exact, W_FLOOR)
            if np.any(w != w_exact):
                clamped += 1
                lu, p, lam_plus, mu_t, D = merit_dir(w)
            mu = mu_t
            if D < 0.0:
                ut, s = full_or_soc(lu, p, mu, D)
                if ut is not None:
                    accepted, soc_taken = True, soc_taken + s
                else:
                    for _ in range(MAX_HALVINGS):
                        alpha *= 0.5
                        backtracks += 1
                        ut = u + alpha * p
                        if dphi(p, mu, alpha, ut) <= ARMIJO * alpha * D:
                            accepted = True
                            break
        if not accepted and h_inf <= LOCAL_H:
            # in the local phase the merit change can fall below the rounding
            # of ||h||_1: take the full step when it reduces the KKT residual
            alpha, ut = 1.0, u + p
            lt = lam + (lam_plus - lam)
            si, hi = _kkt_inf(fam, ut, uhat, lt)
            accepted = max(hi, si / scale) < res
        if not accepted:
            break
        u = ut
        lam = lam + alpha * (lam_plus - lam)
    if best is None:
        h_inf = float(np.abs(fam.h(u)).max(initial=0.0))
        s_inf = _kkt_inf(fam, u, uhat, lam)[0]
        best = (max(h_inf, s_inf / scale), u, lam, it, h_inf, s_inf)
    _, u, lam, it_best, h_inf, s_inf = best
    converged = h_inf <= CONV_TOL and s_inf <= CONV_TOL * scale
    info = dict(iters=it_best, converged=converged, h_inf=h_inf, stat_inf=s_inf,
                objective=0.5 * float((u - uhat) @ (u - uhat)), backtracks=backtracks,
                soc=soc_taken, clamped=clamped, history=history)
    if strict and not converged:
        raise OracleNotConverged(
            f"oracle SQP stopped at ||h||_inf = {h_inf:.3e}, stationarity {s_inf:.3e} "
            f"after {len(history)} evaluations")
    return (u, lam, info) if return_info else (u, lam)


def reduced_hessian_min_eig(fam, u, lam):
    """Smallest eigenvalue of Z^T W Z on null(J) (dense; tiny problems only).
    Positive means the KKT point is a strict local minimizer (second-order
    sufficiency)."""
    import scipy.linalg as sla
    J = fam.jac(u).toarray()
    Z = sla.null_space(J)
    if Z.shape[1] == 0:
        return np.inf
    W = np.diag(_hess_diag(fam, u, lam))
    return float(np.linalg.eigvalsh(Z.T @ W @ Z).min())


def adjoint_sample(fam, u, lam, grad_u, basis="spectral"):
    """d(u*)/d(u_hat)^T grad_u at the KKT point (u, lam).  The 2D diffusion +
    energy family is differentiated in its spectral form (the KKT matrix of
    the rotated problem is the rotated KKT matrix)."""
    sf = _spectral_form(fam, basis)
    if sf is not None:
        k = (fam.nt - 1) * fam.np_
        lv = np.concatenate([sf.to_spectral(lam[:k]), lam[k:]])
        gv = adjoint_sample(sf, sf.to_spectral(u), lv, sf.to_spectral(grad_u), basis="physical")
        return sf.from_spectral(gv)
    n, m = fam.n, fam.m
    g = np.asarray(grad_u, dtype=np.float64).reshape(-1)
    if m == 0:
        return g.copy()
    J = fam.jac(u)
    lu = _kkt_lu(J, _hess_diag(fam, u, lam))
    sol = lu.solve(np.concatenate([g, np.zeros(m)]))
    return sol[:n]


def project_batch(batch, max_iter=200, indices=None, strict=True):
    """Project every sample of a synthgen Batch.  Returns packed (u, lam, iters)."""
    idx = range(len(batch)) if indices is None else indices
    u_out = np.array(batch.uhat, copy=True)
    lam_out = np.zeros(batch.total_rows)
    iters = np.zeros(len(batch), dtype=np.int32)
    for s in idx:
        smp = batch.samples[s]
        fam = family_of(smp)
        u, lam, info = project_sample(fam, smp.uhat.reshape(-1), max_iter=max_iter,
                                      return_info=True, strict=strict)
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
