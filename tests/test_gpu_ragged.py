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


def _fixed_ragged_indices(b):
    """Two Burgers samples of every Nx (the first in batch order, preferring
    short time spans), plus mass + IC and Fisher-KPP samples on the narrow
    (Nx <= 128) and wide (Nx = 192, 256) slab kernels."""
    pick = []
    for nx in synthgen.RAGGED_NX:
        cand = [i for i, s in enumerate(b.samples) if s.family == synthgen.F3_BURGERS_LF and s.nx == nx]
        cand.sort(key=lambda i: (b.samples[i].nt, i))
        pick += cand[:2]
    # one long Burgers sample at the widest band
    pick.append(next(i for i, s in enumerate(b.samples)
                     if s.family == synthgen.F3_BURGERS_LF and s.nx == 256 and s.nt == 128))
    for fam in (synthgen.F1_MASS_IC, synthgen.F2_FISHER_KPP):
        for nx in (64, 128, 192, 256):
            pick.append(next(i for i, s in enumerate(b.samples) if s.family == fam and s.nx == nx))
    return sorted(pick)


@pytest.mark.parametrize("prec,tol,lam_tol", [(snap.PREC_FP64, 1e-10, 1e-8),
                                              (snap.PREC_MIXED, 1e-6, 1e-4)])
def test_ragged_full_config_fixed_samples(prec, tol, lam_tol):
    # the 1024-sample ragged workload in both precisions: every sample
    # converged and feasible by the oracle's evaluator, and a fixed list of
    # samples covering every band class and both slab kernels equal to the
    # oracle's point
    from gpu_helpers import check_samples
    b = synthgen.make("ragged")
    res = gpu_project(b, snap.Options(precision=prec))
    assert (res["stats"]["status"] == 0).all()
    hv = max_violation(b, res["u_np"])
    assert hv.max() <= 1e-8
    check_samples(b, res, _fixed_ragged_indices(b), tol, lam_tol)


def test_ragged_adjoint_central_differences():
    # 16 samples of the ragged workload (at least 5 per family), two random
    # unit directions each: <g, (P(u_hat + eps w) - P(u_hat - eps w)) / 2eps>
    # against <VJP(g), w>, FP64 forwards run to 1e-12 (the last Newton step squares
    # the error, so the forwards' own error stays far below eps * 1e-6)
    import copy
    b = synthgen.make("ragged")
    rng = np.random.default_rng(16)
    chosen = []
    for fam in (synthgen.F1_MASS_IC, synthgen.F2_FISHER_KPP, synthgen.F3_BURGERS_LF):
        idx = [i for i, s in enumerate(b.samples) if s.family == fam]
        chosen += list(rng.choice(idx, size=6 if fam == synthgen.F3_BURGERS_LF else 5, replace=False))
    base = [b.samples[i] for i in chosen]
    eps = 1e-6
    dirs, pert = [], []
    for s in base:
        for _ in range(2):
            w = rng.standard_normal(s.uhat.shape)
            w /= np.linalg.norm(w)
            dirs.append(w)
            for sign in (1.0, -1.0):
                p = copy.copy(s)
                p.uhat = s.uhat + sign * eps * w
                pert.append(p)
    opts = snap.Options(tol_h=1e-12, tol_s=1e-12, max_newton=40, flags=snap.FLAG_KEEP_FACTOR)
    bb = synthgen.Batch(base).pack()
    res = gpu_project(bb, opts)
    assert (res["stats"]["status"] == 0).all(), res["stats"]
    grad = synthgen.upstream_grad(bb, seed=3)
    g, st = gpu_backward(res, grad)
    assert (st["status"] == 0).all()
    bp = synthgen.Batch(pert).pack()
    rp = gpu_project(bp, snap.Options(tol_h=1e-12, tol_s=1e-12, max_newton=40))
    assert (rp["stats"]["status"] == 0).all(), rp["stats"]
    for k, s in enumerate(base):
        vo = bb.var_off[k]
        gs = grad[vo:vo + s.n]
        vjp = g[vo:vo + s.n]
        for d in range(2):
            j = 2 * k + d
            up = rp["u_np"][bp.var_off[2 * j]: bp.var_off[2 * j] + s.n]
            um = rp["u_np"][bp.var_off[2 * j + 1]: bp.var_off[2 * j + 1] + s.n]
            fd = (up - um) / (2 * eps)
            lhs = float(gs @ fd)
            rhs = float(vjp @ dirs[j].reshape(-1))
            scale = np.linalg.norm(gs) * max(np.linalg.norm(fd), 1e-300)
            assert abs(lhs - rhs) <= 1e-6 * scale, (chosen[k], s.family, s.nx, s.nt, lhs, rhs)
