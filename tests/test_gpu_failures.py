"""Failure reporting: each per-sample status is produced by a condition set up
from the host (options or input values), and the other samples of the same
call are unaffected.  Nothing here makes a kernel fault: every input is finite
or a NaN the kernels test for, and every loop is bounded by the options."""
import numpy as np
import pytest

import synthgen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2607_00095_amd as snap  # noqa: E402
from gpu_helpers import gpu_backward, gpu_project, oracle_solution, rel_err, to_dev  # noqa: E402

ST_CONVERGED, ST_LS_FAIL, ST_NONFINITE, ST_SINGULAR, ST_FLOOR = 0, 2, 3, 4, 5


def _strong_fisher():
    smp = [s for dt, seed in ((0.45, 1), (0.5, 4), (0.55, 5))
           for s in synthgen.fisher_kpp_batch(batch=4, nx=20, nt=8, seed=seed, dt=dt).samples]
    return synthgen.Batch(smp, name="fisher_kpp").pack()


def test_no_halvings_allowed_reports_line_search_failure():
    # max_ls = 0: a sample whose full Newton step fails the merit test stops
    # with LS_FAIL; the others converge to the oracle's point
    b = _strong_fisher()
    full = gpu_project(b, snap.Options(max_newton=60))
    res = gpu_project(b, snap.Options(max_newton=60, max_ls=0))
    st = res["stats"]["status"]
    assert set(st.tolist()) <= {ST_CONVERGED, ST_LS_FAIL}
    assert (st == ST_LS_FAIL).any()
    assert (full["stats"]["ls_backtracks"][st == ST_LS_FAIL] > 0).all()
    for s in np.flatnonzero(st == ST_CONVERGED):
        vo, smp = b.var_off[s], b.samples[s]
        u_o, _ = oracle_solution(smp)
        assert rel_err(res["u_np"][vo:vo + smp.n], u_o) <= 1e-10


@pytest.mark.parametrize("name,kw", [("burgers_lf", dict(batch=3, nx=16, nt=8)),
                                     ("diff2d_energy", dict(batch=3, n=16, nt=3))])
def test_nonfinite_input_is_reported(name, kw):
    b = synthgen.make(name, **kw)
    b.uhat[b.var_off[1] + 7] = np.nan
    res = gpu_project(b)
    st = res["stats"]["status"]
    assert st[1] == ST_NONFINITE
    assert st[0] == ST_CONVERGED and st[2] == ST_CONVERGED


def test_fisher_adjoint_reports_a_floored_hessian():
    # multipliers whose Hessian 1 + 2 dt rho lam falls below the floor on a
    # slab: the adjoint says its gradient used the floored W
    b = synthgen.fisher_kpp_batch(batch=3, nx=32, nt=10, seed=2)
    res = gpu_project(b)
    lam = res["lam"].clone()
    smp = b.samples[1]
    k0 = int(b.row_off[1]) + smp.nx + 3            # law row 3 of sample 1
    lam[k0] = -1.0 / (smp.dt * smp.p0)             # W = 1 + 2 dt rho lam = -1
    g, st = snap.project_backward(res["plan"], res["u"], lam, res["aux"], res["ws"],
                                  to_dev(synthgen.upstream_grad(b, seed=1)))
    torch.cuda.synchronize()
    status = snap.stats_to_numpy(st, len(b))["status"]
    assert status.tolist() == [ST_CONVERGED, ST_FLOOR, ST_CONVERGED]


def test_burgers_adjoint_reports_a_floored_hessian():
    b = synthgen.burgers_batch(batch=2, nx=16, nt=6, seed=3)
    res = gpu_project(b)
    lam = res["lam"].clone()
    smp = b.samples[0]
    q = 0.5 * smp.dt / smp.dx
    ro = int(b.row_off[0])
    # a ramp in x on step 2: W = 1 + q (lam(x-1) - lam(x+1)) = 1 - 2 q L at interior x
    L = 2.0 / q
    lam[ro + 2 * smp.nx: ro + 3 * smp.nx] = torch.arange(smp.nx, dtype=torch.float64, device="cuda") * L
    g, st = snap.project_backward(res["plan"], res["u"], lam, res["aux"], res["ws"],
                                  to_dev(synthgen.upstream_grad(b, seed=1)))
    torch.cuda.synchronize()
    status = snap.stats_to_numpy(st, len(b))["status"]
    assert status.tolist() == [ST_FLOOR, ST_CONVERGED]


def test_diff2d_adjoint_reports_an_indefinite_reduced_hessian():
    # energy multipliers of -1 on every frame: W = -1, every mode's reduced
    # Hessian is negative and the elimination does not exist
    b = synthgen.diff2d_batch(batch=2, n=16, nt=3, seed=4)
    res = gpu_project(b)
    lam = res["lam"].clone()
    smp = b.samples[1]
    e0 = int(b.row_off[1]) + (smp.nt - 1) * smp.nx * smp.ny
    lam[e0:e0 + smp.nt] = -1.0
    g, st = snap.project_backward(res["plan"], res["u"], lam, res["aux"], res["ws"],
                                  to_dev(synthgen.upstream_grad(b, seed=1)))
    torch.cuda.synchronize()
    status = snap.stats_to_numpy(st, len(b))["status"]
    assert status.tolist() == [ST_CONVERGED, ST_SINGULAR]
