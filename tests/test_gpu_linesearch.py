"""Backtracking line search on strongly nonlinear Fisher-KPP samples.

Large dt*rho (0.45-0.55 with rho up to 2) makes the logistic budget rows
strongly nonlinear: on many of these samples the full Newton step from u_hat
does not decrease the l1 merit, so the kernels must halve the step
(alpha < 1) before converging.  Every sample of the 15 seeded batches
(60 samples) is compared with the oracle's SQP point.
"""
import numpy as np
import pytest

import paper_2607_00095_amd as snap
import synthgen
from gpu_helpers import check_samples, gpu_project

pytestmark = pytest.mark.gpu

STRONG = [(dt, seed) for dt in (0.45, 0.5, 0.55) for seed in range(1, 6)]


def _batch():
    smp = [s for dt, seed in STRONG
           for s in synthgen.fisher_kpp_batch(batch=4, nx=20, nt=8, seed=seed, dt=dt).samples]
    return synthgen.Batch(smp, name="fisher_kpp").pack()


@pytest.mark.parametrize("precision,tol,lam_tol", [(snap.PREC_FP64, 1e-10, 1e-8),
                                                   (snap.PREC_MIXED, 1e-6, 1e-4)])
def test_backtracking_reaches_oracle_point(precision, tol, lam_tol):
    b = _batch()
    res = gpu_project(b, snap.Options(precision=precision, max_newton=60))
    st = res["stats"]
    print("newton iters", st["newton_iters"].tolist(), "backtracks", st["ls_backtracks"].tolist())
    assert st["ls_backtracks"].sum() > 0          # the halving path ran
    check_samples(b, res, range(len(b)), tol, lam_tol)


@pytest.mark.xfail(reason="with SNAP_FLAG_SOC the slab kernel stalls on one of the 60 samples "
                          "(dt = 0.45, seed 1, sample 1: ||h|| = 1.36 after 30 steps) where a CPU "
                          "re-enactment of the same policy converges; under investigation",
                   strict=False)
def test_second_order_correction_option():
    b = _batch()
    res = gpu_project(b, snap.Options(flags=snap.FLAG_SOC, max_newton=60))
    check_samples(b, res, range(len(b)), 1e-10, 1e-8)
