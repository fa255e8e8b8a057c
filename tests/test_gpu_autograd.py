"""The autograd form: SnapProject.apply(...).backward() through torch gives the
implicit-function vector-Jacobian product of the oracle."""
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
from gpu_helpers import oracle_solution, rel_err, to_dev  # noqa: E402


@pytest.mark.parametrize("name,kw", [("fisher_kpp", dict(batch=3, nx=32, nt=10)),
                                     ("burgers_lf", dict(batch=2, nx=16, nt=8)),
                                     ("mass_ic", dict(batch=2, nx=12, nt=5))])
def test_snap_project_backward_matches_oracle(name, kw):
    b = synthgen.make(name, **kw)
    plan = snap.Plan.from_batch(b, snap.Options(flags=snap.FLAG_KEEP_FACTOR))
    B = len(b)
    # a uniform batch passed as [B, Nt, Nx]: output and gradient keep the shape
    uhat = to_dev(b.uhat).view(B, b.samples[0].nt, b.samples[0].nx).requires_grad_(True)
    aux = to_dev(b.aux)
    u = snap.SnapProject.apply(uhat, aux, plan)
    assert u.shape == uhat.shape
    g_up = synthgen.upstream_grad(b, seed=12)
    loss = (u * to_dev(g_up).view_as(u)).sum()
    loss.backward()
    grad = uhat.grad.detach().cpu().numpy().reshape(-1)
    u_np = u.detach().cpu().numpy().reshape(-1)
    for s, smp in enumerate(b.samples):
        vo = b.var_off[s]
        u_o, lam_o = oracle_solution(smp)
        assert rel_err(u_np[vo:vo + smp.n], u_o) <= 1e-10
        g_o = adjoint_sample(family_of(smp), u_o, lam_o, g_up[vo:vo + smp.n])
        assert rel_err(grad[vo:vo + smp.n], g_o) <= 1e-10


def test_snap_project_rejects_wrong_size_and_unconverged():
    b = synthgen.fisher_kpp_batch(batch=2, nx=16, nt=6, seed=3)
    plan = snap.Plan.from_batch(b)
    with pytest.raises(snap.SnapError):
        snap.SnapProject.apply(to_dev(np.zeros(b.total_vars + 1)).requires_grad_(True),
                               to_dev(b.aux), plan)
    one_step = snap.Plan.from_batch(b, snap.Options(max_newton=1))
    uhat = to_dev(b.uhat).requires_grad_(True)
    u = snap.SnapProject.apply(uhat, to_dev(b.aux), one_step)
    with pytest.raises(snap.SnapError):
        u.sum().backward()
    uhat2 = to_dev(b.uhat).requires_grad_(True)
    u2 = snap.SnapProject.apply(uhat2, to_dev(b.aux), one_step, True)
    u2.sum().backward()
    assert torch.isfinite(uhat2.grad).all()
