"""HIP-graph replay of the launch sequence (SNAP_FLAG_GRAPH) against direct launches.

Every replay runs on new input values written into the same buffers, with the
program's own eager work and synchronizations in between, and must reproduce
the direct (eager) call bit for bit: the graph holds exactly the launches the
eager path makes.
"""
import numpy as np
import pytest
import torch

import paper_2607_00095_amd as snap
import synthgen
from gpu_helpers import to_dev

pytestmark = pytest.mark.gpu

CASES = [
    ("fisher_kpp", dict(batch=6, nx=40, nt=12)),
    ("burgers_lf", dict(batch=3, nx=16, nt=8)),
    ("ragged", dict(batch=12)),
]


@pytest.mark.parametrize("name,kw", CASES)
@pytest.mark.parametrize("precision", [snap.PREC_FP64, snap.PREC_MIXED])
def test_graph_replays_equal_eager(name, kw, precision):
    # one layout (the plan's), new values per replay: seeded perturbations of u_hat
    b0 = synthgen.make(name, **kw)
    batches = []
    for s in (11, 12, 13):
        b = synthgen.make(name, **kw)
        b.uhat = b.uhat + 0.01 * np.random.default_rng(s).standard_normal(b.uhat.shape)
        batches.append(b)
    flags = snap.FLAG_GRAPH | snap.FLAG_KEEP_FACTOR
    plan = snap.Plan.from_batch(b0, snap.Options(precision=precision, flags=flags))
    stream = torch.cuda.Stream()
    uhat = to_dev(b0.uhat)
    aux = to_dev(b0.aux)
    u = torch.empty(max(plan.total_vars, 1), dtype=torch.float64, device="cuda")
    lam = torch.empty(max(plan.total_rows, 1), dtype=torch.float64, device="cuda")
    st = torch.empty(max(plan.batch, 1) * 32, dtype=torch.uint8, device="cuda")
    ws = plan.new_workspace()
    gu = torch.empty_like(u)
    gst = torch.empty_like(st)
    for rep, b in enumerate(batches + batches[:1]):
        assert b.total_vars == b0.total_vars and len(b.aux) == len(b0.aux)
        # eager work of the program itself between replays
        uhat.copy_(to_dev(b.uhat))
        aux.copy_(to_dev(b.aux))
        junk = torch.randn(1000, device="cuda").sum()
        torch.cuda.synchronize()
        with torch.cuda.stream(stream):
            snap.project(plan, uhat, aux, ws, u, lam, st, stream=stream)
            grad = to_dev(synthgen.upstream_grad(b, seed=rep))
            snap.project_backward(plan, u, lam, aux, ws, grad, gu, gst, stream=stream)
        stream.synchronize()
        assert torch.isfinite(junk)
        # the same call without the graph
        ref_plan = snap.Plan.from_batch(b, snap.Options(precision=precision,
                                                       flags=snap.FLAG_KEEP_FACTOR))
        ru, rl, rs, rws = snap.project(ref_plan, to_dev(b.uhat), to_dev(b.aux))
        rg, _ = snap.project_backward(ref_plan, ru, rl, to_dev(b.aux), rws, grad)
        torch.cuda.synchronize()
        n, m = b.total_vars, b.total_rows
        assert torch.equal(u[:n], ru[:n]), f"replay {rep}: u differs"
        assert torch.equal(lam[:m], rl[:m]), f"replay {rep}: lambda differs"
        assert torch.equal(gu[:n], rg[:n]), f"replay {rep}: adjoint differs"
        s = snap.stats_to_numpy(st, len(b))
        assert (s["status"] == 0).all()


def test_graph_recaptures_when_buffers_change():
    # a banded batch: its call is a launch sequence, so it runs from the graph
    # (a single slab-row launch runs directly)
    b = synthgen.make("burgers_lf", batch=2, nx=16, nt=8)
    plan = snap.Plan.from_batch(b, snap.Options(flags=snap.FLAG_GRAPH))
    stream = torch.cuda.Stream()
    outs = []
    for _ in range(2):   # fresh output buffers each time: new pointers, new capture
        with torch.cuda.stream(stream):
            u, lam, st, ws = snap.project(plan, to_dev(b.uhat), to_dev(b.aux), stream=stream)
        stream.synchronize()
        outs.append(u[: b.total_vars].clone())
    ref = snap.project(snap.Plan.from_batch(b), to_dev(b.uhat), to_dev(b.aux))[0]
    torch.cuda.synchronize()
    for o in outs:
        assert torch.equal(o, ref[: b.total_vars])


def test_graph_on_null_stream_runs_directly():
    b = synthgen.make("fisher_kpp", batch=3, nx=24, nt=8)
    plan = snap.Plan.from_batch(b, snap.Options(flags=snap.FLAG_GRAPH))
    u = snap.project(plan, to_dev(b.uhat), to_dev(b.aux))[0]   # current (null) stream
    ref = snap.project(snap.Plan.from_batch(b), to_dev(b.uhat), to_dev(b.aux))[0]
    torch.cuda.synchronize()
    assert np.array_equal(u.cpu().numpy()[: b.total_vars], ref.cpu().numpy()[: b.total_vars])
