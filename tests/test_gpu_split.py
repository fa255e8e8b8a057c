"""GPU parity of the two-sided band factorization: two workgroups per sample
factor the Schur band from both ends toward a separator of BB block rows,
which a third sweep factors last.  Checked against the oracle (forward and
adjoint, with and without a kept factor) and against the one-sided
factorization of the same batch."""
import numpy as np
import pytest

import synthgen
from oracle.families import family_of
from oracle.kkt import adjoint_sample

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2607_00095_amd as snap  # noqa: E402
from gpu_helpers import check_samples, gpu_backward, gpu_project, oracle_solution, rel_err  # noqa: E402

SPLIT = 64          # class offset of the two-sided form


def _dt(nx):
    return 1e-3 * min(1.0, (128.0 / nx) ** 2)


def _band_bb(nx):
    need = -(-(nx + 2) // 16)
    return next(b for b in (13, 17) if b >= need)


def _forced(b, options):
    """Plan with the two-sided class on its one band group."""
    plan = snap.Plan.from_batch(b, options)
    bb = _band_bb(b.samples[0].nx)
    assert SPLIT + bb in plan.group_classes(0), plan.group_classes(0)
    plan.set_group_class(0, SPLIT + bb)
    assert "two-sided" in plan.describe()
    return plan


def _check_adjoint(b, res, grad, tol):
    g, st = gpu_backward(res, grad)
    assert (st["status"] == 0).all(), st["status"]
    for s, smp in enumerate(b.samples):
        vo = b.var_off[s]
        u_o, lam_o = oracle_solution(smp)
        g_o = adjoint_sample(family_of(smp), u_o, lam_o, grad[vo:vo + smp.n])
        assert rel_err(g[vo:vo + smp.n], g_o) <= tol, (s, rel_err(g[vo:vo + smp.n], g_o))
    return g


# short bands with the form forced: parts of a few BB block rows; BB = 13
# and 17; 200 x 8 and 250 x 6 end in a partial block (m % 16 != 0)
FORCED = [(192, 5), (256, 5), (200, 8), (250, 6)]


@pytest.mark.parametrize("nx,nt", FORCED)
@pytest.mark.parametrize("keep", [True, False])
def test_two_sided_matches_oracle(nx, nt, keep):
    b = synthgen.burgers_batch(batch=2, nx=nx, nt=nt, dt=_dt(nx), seed=13 * nx + nt)
    opts = snap.Options(flags=snap.FLAG_KEEP_FACTOR if keep else 0)
    res = gpu_project(b, plan=_forced(b, opts))
    check_samples(b, res, [0, 1], 1e-10, 1e-8)
    # the adjoint reuses the kept two-sided factor, or factors again in the
    # two-sided form
    _check_adjoint(b, res, synthgen.upstream_grad(b, seed=nx + nt), 1e-10)


def test_small_groups_take_the_wider_shapes():
    # at most one sample per CU: two-sided at BB >= 13, 8 wavefronts at BB <= 9;
    # a group larger than the machine keeps the one-sided 4-wavefront default
    small = snap.Plan.from_batch(synthgen.burgers_batch(batch=4, nx=192, nt=9, dt=_dt(192), seed=1))
    assert "two-sided" in small.describe()
    b9 = snap.Plan.from_batch(synthgen.burgers_batch(batch=4, nx=128, nt=9, seed=1))
    assert "class 41, 8 wavefronts" in b9.describe(), b9.describe()
    big = snap.Plan.from_batch(synthgen.burgers_batch(batch=300, nx=128, nt=3, seed=1))
    assert "class 9, 4 wavefronts" in big.describe(), big.describe()


@pytest.mark.parametrize("nx,nt", [(192, 48), (256, 45)])
def test_two_sided_is_the_default_on_long_wide_bands(nx, nt):
    # 564 and 704 block rows: at least 40 BB, where the form is the default
    b = synthgen.burgers_batch(batch=2, nx=nx, nt=nt, dt=_dt(nx), seed=nx * nt)
    res = gpu_project(b, snap.Options(flags=snap.FLAG_KEEP_FACTOR))
    assert "two-sided" in res["plan"].describe()
    check_samples(b, res, [0, 1], 1e-10, 1e-8)
    _check_adjoint(b, res, synthgen.upstream_grad(b, seed=3), 1e-10)


@pytest.mark.parametrize("nx,nt", [(192, 9), (256, 12)])
def test_two_sided_agrees_with_one_sided(nx, nt):
    # the same Newton iteration with the rows eliminated in another order:
    # iterates agree to rounding, the iteration counts exactly
    b = synthgen.burgers_batch(batch=3, nx=nx, nt=nt, dt=_dt(nx), seed=nx + 7 * nt)
    opts = snap.Options(flags=snap.FLAG_KEEP_FACTOR)
    plan_one = snap.Plan.from_batch(b, opts)
    plan_one.set_group_class(0, _band_bb(nx))
    one = gpu_project(b, plan=plan_one)
    assert "two-sided" not in one["plan"].describe()
    two = gpu_project(b, plan=_forced(b, opts))
    np.testing.assert_array_equal(one["stats"]["newton_iters"], two["stats"]["newton_iters"])
    for s, smp in enumerate(b.samples):
        vo, ro = b.var_off[s], b.row_off[s]
        assert rel_err(two["u_np"][vo:vo + smp.n], one["u_np"][vo:vo + smp.n]) <= 1e-12
        assert rel_err(two["lam_np"][ro:ro + smp.m], one["lam_np"][ro:ro + smp.m]) <= 1e-10
    grad = synthgen.upstream_grad(b, seed=5)
    g1, _ = gpu_backward(one, grad)
    g2, _ = gpu_backward(two, grad)
    assert rel_err(g2, g1) <= 1e-11


@pytest.mark.parametrize("nx,nt", [(192, 5), (256, 9)])
def test_two_sided_mixed_precision(nx, nt):
    # float32 factor: the Newton solve refines in the local phase and the
    # adjoint to working precision, with one workgroup sweeping all three
    # parts of the two-sided factor
    b = synthgen.burgers_batch(batch=2, nx=nx, nt=nt, dt=_dt(nx), seed=5 * nx + nt)
    opts = snap.Options(precision=snap.PREC_MIXED, flags=snap.FLAG_KEEP_FACTOR)
    res = gpu_project(b, plan=_forced(b, opts))
    check_samples(b, res, [0, 1], 1e-6, 1e-4)
    _check_adjoint(b, res, synthgen.upstream_grad(b, seed=11), 1e-6)
    # the adjoint refines to working precision: refinement rounds ran
    _, st = gpu_backward(res, synthgen.upstream_grad(b, seed=11))
    assert st["refine_steps"].sum() > 0
    # without a kept factor the adjoint factors again in float32
    res2 = gpu_project(b, plan=_forced(b, snap.Options(precision=snap.PREC_MIXED)))
    _check_adjoint(b, res2, synthgen.upstream_grad(b, seed=11), 1e-6)


def test_mixed_two_sided_default_on_long_wide_bands():
    b = synthgen.burgers_batch(batch=1, nx=256, nt=45, dt=_dt(256), seed=2)
    res = gpu_project(b, snap.Options(precision=snap.PREC_MIXED))
    assert "two-sided" in res["plan"].describe()
    check_samples(b, res, [0], 1e-6, 1e-4)


@pytest.mark.parametrize("prec", [snap.PREC_FP64, snap.PREC_MIXED])
def test_two_sided_refinement_rounds_match_one_sided(prec):
    # the first refinement round of a two-sided step adds its correction to
    # the step in place (the backward sweeps read and write the same vector);
    # a round that lost the step would leave a residual as large as before and
    # cost extra rounds, so the two forms refine about equally often
    b = synthgen.burgers_batch(batch=2, nx=256, nt=45, dt=_dt(256), seed=21)
    opts = snap.Options(precision=prec)
    two = gpu_project(b, opts)
    assert "two-sided" in two["plan"].describe()
    plan_one = snap.Plan.from_batch(b, opts)
    plan_one.set_group_class(0, 17)
    one = gpu_project(b, plan=plan_one)
    assert "two-sided" not in one["plan"].describe()
    assert (two["stats"]["status"] == 0).all() and (one["stats"]["status"] == 0).all()
    r2, r1 = two["stats"]["refine_steps"], one["stats"]["refine_steps"]
    assert (r2 <= r1 + two["stats"]["newton_iters"]).all(), (r2, r1)
