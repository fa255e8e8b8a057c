"""Shared helpers for the GPU parity tests (run the HIP library through the C ABI)."""
import numpy as np
import torch

import paper_2607_00095_amd as snap


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def gpu_project(batch, options=None):
    plan = snap.Plan.from_batch(batch, options or snap.Options())
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
