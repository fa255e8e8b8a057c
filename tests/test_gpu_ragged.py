"""Ragged batches: mixed families and grid sizes in one call, each sample equal
to its own projection (batch independence) and to the oracle."""
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


def _small_ragged(seed=11, n=24):
    return synthgen.ragged_batch(batch=n, seed=seed, nx_choices=(16, 24, 40, 64),
                                 nt_choices=(4, 9, 16))


@pytest.mark.parametrize("prec,tol", [(snap.PREC_FP64, 1e-10), (snap.PREC_MIXED, 1e-6)])
def test_ragged_matches_oracle(prec, tol):
    b = _small_ragged()
    res = gpu_project(b, snap.Options(precision=prec))
    assert (res["stats"]["status"] == 0).all(), res["stats"]
    hv = max_violation(b, res["u_np"])
    assert hv.max() <= 1e-8
    for s, smp in enumerate(b.samples):
        u_o, _ = project_sample(family_of(smp), smp.uhat.reshape(-1))
        vo = b.var_off[s]
        assert rel_err(res["u_np"][vo:vo + smp.n], u_o) <= tol, (s, smp.family, smp.nx, smp.nt)


def test_ragged_equals_individual_projection():
    b = _small_ragged(seed=5, n=10)
    res = gpu_project(b)
    for s in (0, 4, 9):
        one = synthgen.Batch([b.samples[s]]).pack()
        r1 = gpu_project(one)
        vo = b.var_off[s]
        np.testing.assert_array_equal(res["u_np"][vo:vo + b.samples[s].n], r1["u_np"])


def test_ragged_backward_matches_oracle():
    b = _small_ragged(seed=8, n=9)
    res = gpu_project(b, snap.Options(flags=snap.FLAG_KEEP_FACTOR))
    grad = synthgen.upstream_grad(b, seed=2)
    g, st = gpu_backward(res, grad)
    assert (st["status"] == 0).all()
    for s, smp in enumerate(b.samples):
        vo = b.var_off[s]
        fam = family_of(smp)
        u_o, lam_o = project_sample(fam, smp.uhat.reshape(-1))
        g_o = adjoint_sample(fam, u_o, lam_o, grad[vo:vo + smp.n])
        assert rel_err(g[vo:vo + smp.n], g_o) <= 1e-9, (s, smp.family)


def test_ragged_full_config_sampled():
    # the 1024-sample ragged workload, mixed precision, sampled against the oracle
    b = synthgen.make("ragged")
    res = gpu_project(b, snap.Options(precision=snap.PREC_MIXED))
    assert (res["stats"]["status"] == 0).all()
    hv = max_violation(b, res["u_np"], indices=range(0, 1024, 7))
    assert hv[::7].max() <= 1e-8
    rng = np.random.default_rng(0)
    for s in rng.choice(1024, size=6, replace=False):
        smp = b.samples[s]
        if smp.family == synthgen.F3_BURGERS_LF and smp.nx * smp.nt > 128 * 64:
            continue      # keep the oracle part within seconds
        u_o, _ = project_sample(family_of(smp), smp.uhat.reshape(-1))
        vo = b.var_off[s]
        assert rel_err(res["u_np"][vo:vo + smp.n], u_o) <= 1e-6, (s, smp.family, smp.nx, smp.nt)
