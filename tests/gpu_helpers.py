"""Shared helpers for the GPU parity tests (run the HIP library through the C ABI)."""
import numpy as np
import torch

import paper_2607_00095_amd as snap


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def gpu_project(batch, options=None, plan=None):
    plan = plan or snap.Plan.from_batch(batch, options or snap.Options())
    uhat = to_dev(batch.uhat)
    aux = to_dev(batch.aux)
    u, lam, st, ws = snap.project(plan, uhat, aux)
    torch.cuda.synchronize()
    stats = snap.stats_to_numpy(st, len(batch))
    return dict(plan=plan, u=u, lam=lam, ws=ws, aux=aux, uhat=uhat,
                u_np=u.cpu().numpy()[: batch.total_vars], lam_np=lam.cpu().numpy()[: batch.total_rows],
                stats=stats)


def gpu_backward(res, grad):
    g, st = snap.project_backward(res["plan"], res["u"], res["lam"], res["aux"], res["ws"], to_dev(grad))
    torch.cuda.synchronize()
    return g.cpu().numpy()[: grad.size], snap.stats_to_numpy(st, res["plan"].batch)


def rel_err(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


_ORACLE_CACHE = {}


def oracle_solution(smp):
    """(u, lam) of the CPU oracle for one synthgen Sample, cached by content."""
    from oracle.families import family_of
    from oracle.kkt import project_sample
    key = (int(smp.family), smp.nx, smp.ny, smp.nt, smp.dt, smp.p0, smp.p1,
           smp.uhat.tobytes(), None if smp.aux is None else smp.aux.tobytes())
    if key not in _ORACLE_CACHE:
        _ORACLE_CACHE[key] = project_sample(family_of(smp), smp.uhat.reshape(-1))
    return _ORACLE_CACHE[key]


def max_abs_rel(a, b):
    """Element-wise agreement: max |a - b| relative to max |b|."""
    return float(np.abs(a - b).max(initial=0.0) / max(np.abs(b).max(initial=0.0), 1e-300))


def check_samples(batch, res, indices, u_tol, lam_tol, h_tol=1e-8):
    """Per-sample parity of a GPU result against the oracle: status, oracle-
    evaluated feasibility, relative 2-norm and element-wise max error of u,
    and the multipliers.  Returns the worst relative u error."""
    from oracle.metric import max_violation
    indices = list(indices)
    st = res["stats"]
    assert (st["status"][indices] == 0).all(), st[indices]
    hv = max_violation(batch, res["u_np"], indices=indices)
    assert hv[indices].max() <= h_tol, hv[indices].max()
    worst = 0.0
    for s in indices:
        smp = batch.samples[s]
        u_o, lam_o = oracle_solution(smp)
        vo, ro = batch.var_off[s], batch.row_off[s]
        u_g = res["u_np"][vo:vo + smp.n]
        e = rel_err(u_g, u_o)
        ea = max_abs_rel(u_g, u_o)
        worst = max(worst, e, ea)
        assert e <= u_tol and ea <= u_tol, (s, smp.family, smp.nx, smp.nt, e, ea)
        lam_g = res["lam_np"][ro:ro + smp.m]
        assert np.abs(lam_g - lam_o).max() <= lam_tol * (1 + np.abs(lam_o).max()), \
            (s, np.abs(lam_g - lam_o).max())
    return worst
