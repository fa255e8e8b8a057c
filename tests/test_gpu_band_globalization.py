"""Globalization of the banded family on the GPU: Burgers samples whose u_hat
carries large noise (amplitude 3-10 against fields of size 1, time steps up
to 0.01) are far from the constraint manifold, so the full Newton step from
(u_hat, 0) often fails the l1-merit test and the Hessian diagonal W falls
below its floor.  The kernels must backtrack and converge.

Far from the manifold the point reached depends on the path: the oracle
first tries the step with the exact (possibly indefinite) W and second-
order corrections, the band kernels always take the floored W.  Where the
two reach different local minimizers, both are valid results of the method
(a strict local minimizer reached from (u_hat, 0)), so a sample passes when
it matches the oracle's point, or when the GPU point is itself a KKT point
with a positive definite reduced Hessian; most samples must match."""
import numpy as np
import pytest

import paper_2607_00095_amd as snap
import synthgen
from gpu_helpers import gpu_project, oracle_solution, rel_err
from oracle.families import family_of
from oracle.kkt import reduced_hessian_min_eig
from oracle.metric import max_violation


def _check(b, res, tol, lam_tol):
    st = res["stats"]
    assert (st["status"] == 0).all(), st["status"]
    hv = max_violation(b, res["u_np"])
    assert hv.max() <= 1e-8, hv.max()
    same = 0
    for s, smp in enumerate(b.samples):
        vo, ro = b.var_off[s], b.row_off[s]
        u, lam = res["u_np"][vo:vo + smp.n], res["lam_np"][ro:ro + smp.m]
        u_o, lam_o = oracle_solution(smp)
        if rel_err(u, u_o) <= tol:
            assert np.abs(lam - lam_o).max() <= lam_tol * (1 + np.abs(lam_o).max()), s
            same += 1
            continue
        # another local minimizer: stationarity, and second-order sufficiency
        fam = family_of(smp)
        uh = smp.uhat.reshape(-1)
        stat = np.abs(u - uh + fam.jac(u).T @ lam).max()
        assert stat <= 10 * tol * (1 + np.abs(uh).max()), (s, stat)
        assert reduced_hessian_min_eig(fam, u, lam) > 0.0, s
        print("sample %d: another local minimizer, objective %.6f (oracle %.6f)"
              % (s, 0.5 * np.sum((u - uh) ** 2), 0.5 * np.sum((u_o - uh) ** 2)))
    assert 2 * same >= len(b), same

pytestmark = pytest.mark.gpu

# (nx, nt, dt, noise amplitude): every batch of four makes the oracle
# backtrack, floor W or take a correction on some of its samples
CASES = [(32, 8, 0.01, 3.0), (24, 8, 0.01, 4.0), (16, 8, 0.01, 10.0), (192, 5, 0.003, 3.0)]


def _noisy(nx, nt, dt, amp, seed=21, batch=4):
    b = synthgen.burgers_batch(batch=batch, nx=nx, nt=nt, dt=dt, seed=seed)
    rng = np.random.default_rng(seed + 1)
    for s in b.samples:
        s.uhat = s.uhat + amp * rng.standard_normal(s.uhat.shape)
    return synthgen.Batch(b.samples, name="burgers_lf").pack()


@pytest.mark.parametrize("nx,nt,dt,amp", CASES)
@pytest.mark.parametrize("precision,tol,lam_tol", [(snap.PREC_FP64, 1e-10, 1e-8),
                                                   (snap.PREC_MIXED, 1e-6, 1e-4)])
def test_noisy_burgers_reaches_oracle_point(nx, nt, dt, amp, precision, tol, lam_tol):
    b = _noisy(nx, nt, dt, amp)
    res = gpu_project(b, snap.Options(precision=precision, max_newton=100))
    st = res["stats"]
    print("newton iters", st["newton_iters"].tolist(), "backtracks", st["ls_backtracks"].tolist())
    _check(b, res, tol, lam_tol)


def test_noisy_burgers_backtracks():
    # the halving path of band_step runs on these inputs
    total = 0
    for nx, nt, dt, amp in CASES[:2]:
        res = gpu_project(_noisy(nx, nt, dt, amp), snap.Options(max_newton=100))
        total += int(res["stats"]["ls_backtracks"].sum())
    assert total > 0


def test_noisy_burgers_two_sided():
    # the same globalization with the two-sided factorization (forced on a
    # short 192-wide band)
    b = _noisy(192, 5, 0.003, 3.0)
    plan = snap.Plan.from_batch(b, snap.Options(max_newton=100))
    plan.set_group_class(0, 64 + 13)
    res = gpu_project(b, plan=plan)
    _check(b, res, 1e-10, 1e-8)


@pytest.mark.parametrize("precision,tol,lam_tol", [(snap.PREC_FP64, 1e-10, 1e-8),
                                                   (snap.PREC_MIXED, 1e-6, 1e-4)])
def test_noisy_burgers_second_order_correction(precision, tol, lam_tol):
    # SNAP_FLAG_SOC: band_soc solves S z = h(u + p) with the step's factor and
    # tries u + p - W^{-1} J^T z before halving.  Every sample still
    # converges to a valid point, and the correction changes the iteration on
    # some sample (the path ran)
    changed = 0
    for nx, nt, dt, amp in CASES:
        b = _noisy(nx, nt, dt, amp)
        plain = gpu_project(b, snap.Options(precision=precision, max_newton=100))
        res = gpu_project(b, snap.Options(precision=precision, max_newton=100, flags=snap.FLAG_SOC))
        print("soc newton iters", res["stats"]["newton_iters"].tolist(),
              "plain", plain["stats"]["newton_iters"].tolist())
        _check(b, res, tol, lam_tol)
        changed += int((res["stats"]["newton_iters"] != plain["stats"]["newton_iters"]).sum())
    assert changed > 0


def test_noisy_burgers_second_order_correction_two_sided():
    b = _noisy(192, 5, 0.003, 3.0)
    plan = snap.Plan.from_batch(b, snap.Options(max_newton=100, flags=snap.FLAG_SOC))
    plan.set_group_class(0, 64 + 13)
    res = gpu_project(b, plan=plan)
    _check(b, res, 1e-10, 1e-8)
    print("two-sided soc newton iters", res["stats"]["newton_iters"].tolist())
