"""GPU parity of the banded Burgers path (block-band LDL^T Schur solver) against the oracle."""
import numpy as np
import pytest

import synthgen
from oracle.families import family_of
from oracle.kkt import adjoint_sample, project_sample
from oracle.metric import max_violation

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2607_00095_amd as snap  # noqa: E402
from gpu_helpers import gpu_backward, gpu_project, rel_err  # noqa: E402

H_TOL = 1e-8


def _check(batch, res, indices, u_tol, lam_tol):
    st = res["stats"]
    assert (st["status"][indices] == 0).all(), st[indices]
    hv = max_violation(batch, res["u_np"], indices=indices)
    assert hv[indices].max() <= H_TOL, hv[indices].max()
    worst = 0.0
    for s in indices:
        smp = batch.samples[s]
        u_o, lam_o = project_sample(family_of(smp), smp.uhat.reshape(-1))
        vo, ro = batch.var_off[s], batch.row_off[s]
        e = rel_err(res["u_np"][vo:vo + smp.n], u_o)
        worst = max(worst, e)
        assert e <= u_tol, (s, e)
        lam_g = res["lam_np"][ro:ro + smp.m]
        assert np.abs(lam_g - lam_o).max() <= lam_tol * (1 + np.abs(lam_o).max()), s
    return worst


@pytest.mark.parametrize("nx,nt", [(16, 8), (13, 6), (32, 17), (3, 4), (40, 2)])
def test_burgers_small_fp64(nx, nt):
    b = synthgen.burgers_batch(batch=3, nx=nx, nt=nt, seed=nx * 31 + nt)
    res = gpu_project(b)
    _check(b, res, list(range(len(b))), 1e-10, 1e-8)


@pytest.mark.parametrize("nx,nt", [(64, 32), (128, 16)])
def test_burgers_medium_fp64(nx, nt):
    b = synthgen.burgers_batch(batch=2, nx=nx, nt=nt, seed=nx + nt)
    res = gpu_project(b)
    _check(b, res, [0, 1], 1e-10, 1e-8)


@pytest.mark.parametrize("nx,nt", [(16, 8), (64, 32)])
def test_burgers_mixed(nx, nt):
    b = synthgen.burgers_batch(batch=2, nx=nx, nt=nt, seed=5 * nx + nt)
    res = gpu_project(b, snap.Options(precision=snap.PREC_MIXED))
    _check(b, res, [0, 1], 1e-6, 1e-4)


@pytest.mark.parametrize("prec", [snap.PREC_FP64, snap.PREC_MIXED])
def test_burgers_backward(prec):
    b = synthgen.burgers_batch(batch=2, nx=16, nt=8, seed=77)
    for flags in (0, snap.FLAG_KEEP_FACTOR):
        res = gpu_project(b, snap.Options(precision=prec, flags=flags))
        grad = synthgen.upstream_grad(b, seed=5)
        g, st = gpu_backward(res, grad)
        assert (st["status"] == 0).all()
        for s, smp in enumerate(b.samples):
            vo = b.var_off[s]
            u_o, lam_o = project_sample(family_of(smp), smp.uhat.reshape(-1))
            g_o = adjoint_sample(family_of(smp), u_o, lam_o, grad[vo:vo + smp.n])
            tol = 1e-10 if prec == snap.PREC_FP64 else 1e-6
            assert rel_err(g[vo:vo + smp.n], g_o) <= tol, (flags, s, rel_err(g[vo:vo + smp.n], g_o))


def test_burgers_full_config_sampled():
    # the full Burgers batch (512 x 128 x 128) in the launch configuration bench.py times;
    # the oracle checks a sample of outputs one by one
    b = synthgen.make("burgers_lf")
    res = gpu_project(b)
    st = res["stats"]
    assert (st["status"] == 0).all()
    assert st["h_inf"].max() <= H_TOL
    _check(b, res, [0, 255, 511], 1e-10, 1e-8)


def test_burgers_mixed_full_config_sampled():
    b = synthgen.make("burgers_lf")
    res = gpu_project(b, snap.Options(precision=snap.PREC_MIXED))
    assert (res["stats"]["status"] == 0).all()
    _check(b, res, [3, 300], 1e-6, 1e-4)


# Every band class of the ragged workload: Nx = 64 / 96 / 128 / 192 / 256 give
# block bandwidths BB = 5 / 7 / 9 / 13 / 17.  Each shape runs with every
# launch shape its group offers (one-sided 4 or 8 wavefronts, two-sided).
# Short time spans keep the oracle within seconds.
WIDE = [(96, 6), (192, 5), (256, 4), (96, 33), (256, 9)]


@pytest.mark.parametrize("nx,nt", WIDE)
@pytest.mark.parametrize("prec", [snap.PREC_FP64, snap.PREC_MIXED])
def test_burgers_every_band_class(nx, nt, prec):
    from gpu_helpers import check_samples, oracle_solution
    dt = 1e-3 * min(1.0, (128.0 / nx) ** 2)
    b = synthgen.burgers_batch(batch=2, nx=nx, nt=nt, dt=dt, seed=9 * nx + nt)
    opts = snap.Options(precision=prec, flags=snap.FLAG_KEEP_FACTOR)
    fp64 = prec == snap.PREC_FP64
    grad = synthgen.upstream_grad(b, seed=nx)
    for cls in snap.Plan.from_batch(b, opts).group_classes(0):
        plan = snap.Plan.from_batch(b, opts)
        plan.set_group_class(0, cls)
        res = gpu_project(b, plan=plan)
        check_samples(b, res, [0, 1], 1e-10 if fp64 else 1e-6, 1e-8 if fp64 else 1e-4)
        g, st = gpu_backward(res, grad)
        assert (st["status"] == 0).all()
        for s, smp in enumerate(b.samples):
            vo = b.var_off[s]
            u_o, lam_o = oracle_solution(smp)
            g_o = adjoint_sample(family_of(smp), u_o, lam_o, grad[vo:vo + smp.n])
            assert rel_err(g[vo:vo + smp.n], g_o) <= (1e-10 if fp64 else 1e-6), \
                (cls, s, rel_err(g[vo:vo + smp.n], g_o))


@pytest.mark.parametrize("prec", [snap.PREC_FP64, snap.PREC_MIXED])
def test_burgers_full_config_adjoint_sampled(prec):
    # the full Burgers batch (BB = 9), forward with the factor kept, then the
    # adjoint; two samples against the oracle's dense-KKT adjoint
    from gpu_helpers import oracle_solution
    b = synthgen.make("burgers_lf")
    res = gpu_project(b, snap.Options(precision=prec, flags=snap.FLAG_KEEP_FACTOR))
    assert (res["stats"]["status"] == 0).all()
    grad = synthgen.upstream_grad(b, seed=7)
    g, st = gpu_backward(res, grad)
    assert (st["status"] == 0).all()
    tol = 1e-10 if prec == snap.PREC_FP64 else 1e-6
    for s in (1, 400):
        smp = b.samples[s]
        vo = b.var_off[s]
        u_o, lam_o = oracle_solution(smp)
        g_o = adjoint_sample(family_of(smp), u_o, lam_o, grad[vo:vo + smp.n])
        assert rel_err(g[vo:vo + smp.n], g_o) <= tol, (s, rel_err(g[vo:vo + smp.n], g_o))
