"""Benchmark of the batched constraint projection on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

A step is one forward projection (the whole Newton/SQP hot path: stencil
evaluation, Schur assembly, factorization, solves, line search, convergence
test) of one batch of synthetic samples already resident in HBM.  The default
workload is the ragged batch: 1024 samples mixing the mass + IC, Fisher-KPP
and Burgers flux families on Nx in {64, 96, 128, 192, 256} x Nt in
{32, 64, 128}, FP64.  The same run also times the mixed-precision forward,
the adjoint and the batched form (autotuned launch shapes, HIP-graph replay),
measures the dominant kernel against its roofline with HIP events recorded on
its launch stream (the banded factorization for workloads with Burgers
samples, else the one-launch slab kernel), and times the CPU oracle on a
bounded sample of the same workload.  Prints one JSON line.
"""
import argparse
import hashlib
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import synthgen  # noqa: E402

HBM_PEAK_GBS = 8000.0
H_FEAS = 1e-8

# bytes that one sample must move at minimum: read u_hat and aux, write u,
# lambda and the stats record (float64 everywhere, 32-byte stats)
def algorithmic_bytes(batch):
    tot = 0
    for s in batch.samples:
        tot += 8 * (2 * s.n + s.m + len(s.aux)) + 32
    return tot


KERNEL_SOURCES = {
    "fisher_kpp": "paper_2607_00095_amd/csrc/snap_slab.hip",
    "mass_ic": "paper_2607_00095_amd/csrc/snap_slab.hip",
    "burgers_lf": "paper_2607_00095_amd/csrc/snap_band.hip",
    "ragged": "paper_2607_00095_amd/csrc/snap_band.hip",
    "diff2d_energy": "paper_2607_00095_amd/csrc/snap_spec.hip",
    "burgers_bc": "paper_2607_00095_amd/csrc/snap_bc.hip",
    "burgers_godunov": "paper_2607_00095_amd/csrc/snap_band.hip",
}
# the dominant kernel of each workload; a band factorization launch is one
# band_factor, or (two-sided form, wide bands) a band_split_rhs +
# band_split_factor + band_split_sep sequence timed as one
KERNEL_NAMES = {
    "fisher_kpp": "slab_kernel", "mass_ic": "slab_kernel",
    "burgers_lf": "band_factor", "ragged": "band_factor | band_split_rhs+band_split_factor+band_split_sep",
    "diff2d_energy": "spec_kernel",
    "burgers_bc": "bc_kernel",
    "burgers_godunov": "band_factor",
}
FP64_PEAK_TFLOPS = 78.6


def band_work(batch, iters):
    """Algorithmic work of the banded samples' factorizations and backward
    substitutions in one call: per factorization m * b^2 flop (m rows, half
    bandwidth b = Nx + 2 in the folded row order), per substitution the factor
    band m * (b + 1) entries read once; one of each per Newton step."""
    flops = sbytes = 0.0
    for s, it in zip(batch.samples, iters):
        if int(s.family) not in (3, 6):
            continue
        m, b = s.nx * (s.nt - 1), s.nx + 2
        flops += float(it) * m * b * b
        sbytes += float(it) * m * (b + 1) * 8
    return flops, sbytes


BAND_BBS = (1, 2, 3, 5, 7, 9, 13, 17)


def factor_bytes(batch, elem=8):
    """Bytes of the stored band factor (16x16 blocks, BB+1 per block panel) of
    the batch's banded samples: what one substitution sweep reads."""
    tot = 0
    for s in batch.samples:
        if int(s.family) not in (3, 6):
            continue
        b = s.nx + 2 if s.nt > 2 else 4
        need = (max(b, 4) + 15) // 16
        bb = next(x for x in BAND_BBS if x >= need)
        nb = (s.nx * (s.nt - 1) + 15) // 16
        tot += nb * (bb + 1) * 256 * elem
    return tot


def source_hash(path):
    with open(os.path.join(ROOT, path), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def load_traffic(workload):
    """HBM traffic per launch from committed rocprofv3 counter runs, if they
    were taken on the current kernel source (else None)."""
    p = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    if not os.path.exists(p):
        return None
    with open(p) as f:
        t = json.load(f)
    if t.get("source_sha") != source_hash(KERNEL_SOURCES[workload]):
        return None
    return t.get("bytes_per_launch")


# ------------------------------------------------------------------ CPU oracle
_POOL_BATCH = None   # the batch, rebuilt from its seed in each oracle worker


def _oracle_init(name):
    global _POOL_BATCH
    _POOL_BATCH = synthgen.make(name)


def _oracle_ready(_):
    return _POOL_BATCH is not None


def _oracle_one(idx):
    """The oracle on one sample: its point, or None where its (semismooth)
    Newton iteration stalls without converging (timed all the same)."""
    from oracle.families import family_of
    from oracle.kkt import OracleNotConverged, project_sample
    s = _POOL_BATCH.samples[idx]
    try:
        u, lam = project_sample(family_of(s), s.uhat.reshape(-1))
    except OracleNotConverged:
        u = None
    return idx, u


def cpu_baseline(name, batch, budget_s=15.0, give_up_s=150.0):
    """Samples/s of the CPU oracle on the first samples of the batch, in a
    pool of fresh worker processes (one BLAS thread each); stops taking
    results once the time budget is spent, or when none arrives for
    give_up_s."""
    workers = max(1, min(16, os.cpu_count() or 1))
    saved = {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")}
    for k in saved:
        os.environ[k] = "1"
    try:
        pool = mp.get_context("spawn").Pool(workers, initializer=_oracle_init, initargs=(name,))
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    res = {}
    try:
        pool.map(_oracle_ready, range(workers), chunksize=1)   # workers up, batch built
        print(f"cpu baseline: {workers} oracle workers ready", file=sys.stderr, flush=True)
        t0 = time.perf_counter()
        it = pool.imap(_oracle_one, range(len(batch)), chunksize=1)
        for i in range(len(batch)):
            try:
                idx, u = it.next(timeout=give_up_s)
            except mp.TimeoutError:
                break
            res[idx] = u
            if time.perf_counter() - t0 >= budget_s and len(res) >= workers:
                break
        wall = time.perf_counter() - t0
    finally:
        pool.terminate()
        pool.join()
    count = len(res)
    print(f"cpu baseline: {count} samples in {wall:.1f} s", file=sys.stderr, flush=True)
    return dict(value=count / wall, unit="samples/s", cores=workers, kind="oracle",
                sample=f"first {count} of {len(batch)} samples of the same batch (in order), "
                       f"pool of {workers} processes with one BLAS thread each, {wall:.1f} s wall"), res


# ------------------------------------------------------------------ GPU timing
def time_calls(fn, steps, warmup, stream):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for _ in range(steps):
        fn()
    stop.record(stream)
    torch.cuda.synchronize()
    return start.elapsed_time(stop) / 1e3 / steps   # seconds per call


def launch_seconds(fn, steps, stream):
    """Average duration of one call that is a single kernel launch: a HIP
    event pair on the launch stream around each call (the whole-call timing
    above also counts the host's gaps between calls)."""
    import torch
    pairs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
             for _ in range(steps)]
    torch.cuda.synchronize()
    for e0, e1 in pairs:
        e0.record(stream)
        fn()
        e1.record(stream)
    torch.cuda.synchronize()
    return sum(e0.elapsed_time(e1) for e0, e1 in pairs) / 1e3 / steps


def sweep(args):
    """Forward time of the plain FP64 and mixed forms against batch size, with
    the workload's shapes (seeded samples of the same generator)."""
    import torch
    import paper_2607_00095_amd as snap
    dev = torch.device("cuda", 0)
    stream = torch.cuda.current_stream(dev)
    for B in (1, 8, 32, 128, 512, 2048):
        batch = synthgen.make(args.workload, batch=B)
        uhat = torch.from_numpy(batch.uhat).to(dev)
        aux = torch.from_numpy(batch.aux).to(dev)
        row = {"workload": args.workload, "batch": B}
        for label, prec in (("fp64", snap.PREC_FP64), ("mixed", snap.PREC_MIXED)):
            plan = snap.Plan.from_batch(batch, snap.Options(precision=prec))
            ws = plan.new_workspace()
            u = torch.empty(plan.total_vars, dtype=torch.float64, device=dev)
            lam = torch.empty(max(plan.total_rows, 1), dtype=torch.float64, device=dev)
            st = torch.empty(B * 32, dtype=torch.uint8, device=dev)
            steps = max(2, min(args.steps, 20))
            sec = time_calls(lambda: snap.project(plan, uhat, aux, ws, u, lam, st, stream),
                             steps, max(1, args.warmup), stream)
            ok = int((snap.stats_to_numpy(st, B)["status"] == 0).sum())
            row[label] = {"ms_per_call": sec * 1e3, "samples_per_s": ok / sec, "converged": ok}
            del plan, ws
            torch.cuda.empty_cache()
        print(json.dumps(row), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="ragged", choices=sorted(KERNEL_SOURCES))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--forward-only", action="store_true",
                    help="time the FP64 forward only (for profiler runs)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only copy 512 MiB device-to-device 5 times (calibrates HBM byte counters)")
    ap.add_argument("--sweep", action="store_true",
                    help="forward time against batch size (1 .. 2048) for the workload; one JSON line per size")
    args = ap.parse_args()
    if args.copy_probe:
        import torch
        src = torch.ones(64 * 1024 * 1024, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_each_way": src.numel() * 8, "copies": 5}))
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: every sample is independent and the library has no "
              "multi-GPU path; run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    if args.sweep:
        sweep(args)
        return

    name = args.workload
    spec = dict(synthgen.CONFIGS[name]["kw"])
    batch = synthgen.make(name)
    B = len(batch)

    # the CPU oracle runs first, in worker processes, before anything touches the GPU
    cb = orc = None
    if not args.no_cpu_baseline:
        cb, orc = cpu_baseline(name, batch)

    import torch
    import paper_2607_00095_amd as snap
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream(dev)
    uhat = torch.from_numpy(batch.uhat).to(dev)
    aux = torch.from_numpy(batch.aux).to(dev)

    plan64 = snap.Plan.from_batch(batch, snap.Options())
    ws = plan64.new_workspace()
    u = torch.empty(plan64.total_vars, dtype=torch.float64, device=dev)
    lam = torch.empty(max(plan64.total_rows, 1), dtype=torch.float64, device=dev)
    st = torch.empty(B * 32, dtype=torch.uint8, device=dev)

    def fwd64():
        snap.project(plan64, uhat, aux, ws, u, lam, st, stream)

    banded = any(int(s.family) in (3, 6) for s in batch.samples)

    # timed region: K forward projections of the resident batch
    torch.cuda.synchronize()
    for _ in range(args.warmup):
        fwd64()
    torch.cuda.synchronize()
    if banded:
        # HIP events around every band_factor / band_solve launch, on the
        # stream each is launched on (from a pool the plan preallocates)
        plan64.set_kernel_timing(True)
    t0 = time.perf_counter()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(args.steps):
        fwd64()
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    sec64 = ev0.elapsed_time(ev1) / 1e3 / args.steps

    stats = snap.stats_to_numpy(st, B)
    u_np = u.cpu().numpy()
    from oracle.metric import max_violation   # feasibility re-evaluated by the oracle's h
    hv = max_violation(batch, u_np)
    ok = (stats["status"] == 0) & (hv <= H_FEAS)
    projected = int(ok.sum())
    value = projected / sec64

    out = {
        "metric": "projected samples/sec at ||h||inf<=1e-8 (forward projection, plain FP64)",
        "value": value,
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec64 * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": name, "batch": B, **{k: v for k, v in spec.items() if k != "seed"},
                   "seed": spec.get("seed"), "precision": "fp64"},
        "projected": projected,
        "max_h_inf": float(hv.max()),
        "newton_iters_mean": float(stats["newton_iters"].mean()),
    }

    if not args.forward_only:
        # mixed precision forward
        plan32 = snap.Plan.from_batch(batch, snap.Options(precision=snap.PREC_MIXED))
        ws32 = plan32.new_workspace()
        u32 = torch.empty_like(u)
        st32 = torch.empty_like(st)
        sec32 = time_calls(lambda: snap.project(plan32, uhat, aux, ws32, u32, lam, st32, stream),
                           args.steps, args.warmup, stream)
        s32 = snap.stats_to_numpy(st32, B)
        u32_np = u32.cpu().numpy()
        hv32 = max_violation(batch, u32_np)
        ok32 = (s32["status"] == 0) & (hv32 <= H_FEAS)
        out["mixed"] = {"value": int(ok32.sum()) / sec32, "ms_per_step": sec32 * 1e3,
                        "max_rel_u_vs_fp64": float(np.max([
                            np.linalg.norm(u32_np[o:o + s.n] - u_np[o:o + s.n]) /
                            max(np.linalg.norm(u_np[o:o + s.n]), 1e-300)
                            for s, o in zip(batch.samples, batch.var_off)]))}
        # adjoint (vector-Jacobian product) with the factor kept by the forward
        plank = snap.Plan.from_batch(batch, snap.Options(flags=snap.FLAG_KEEP_FACTOR))
        wsk = plank.new_workspace()
        uk, lk, stk = torch.empty_like(u), torch.empty_like(lam), torch.empty_like(st)
        snap.project(plank, uhat, aux, wsk, uk, lk, stk, stream)
        grad = torch.from_numpy(synthgen.upstream_grad(batch, seed=7)).to(dev)
        gout = torch.empty_like(u)
        stb = torch.empty_like(st)
        secb = time_calls(lambda: snap.project_backward(plank, uk, lk, aux, wsk, grad, gout, stb, stream),
                          args.steps, args.warmup, stream)
        out["backward"] = {"value": B / secb, "ms_per_step": secb * 1e3, "unit": "samples/s"}
        fb = factor_bytes(batch)
        if fb:
            # the adjoint of the banded samples is one forward and one backward
            # substitution sweep over the kept factor: it streams the factor twice
            out["backward"]["factor_stream"] = {
                "bytes": 2 * fb, "achieved": 2 * fb / secb / 1e9, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": 2 * fb / secb / 1e9 / HBM_PEAK_GBS}

        # batched form: launch shapes picked by the plan's autotuner, the whole
        # launch sequence replayed from a HIP graph (needs a non-null stream)
        side = torch.cuda.Stream(dev)
        for label, prec in (("batched_fp64", snap.PREC_FP64), ("batched_mixed", snap.PREC_MIXED)):
            t0b = time.perf_counter()
            planb = snap.Plan.from_batch(batch, snap.Options(
                precision=prec, flags=snap.FLAG_AUTOTUNE | snap.FLAG_GRAPH))
            tune_s = time.perf_counter() - t0b
            wsb = planb.new_workspace()
            ub, stb2 = torch.empty_like(u), torch.empty_like(st)
            with torch.cuda.stream(side):
                secg = time_calls(lambda: snap.project(planb, uhat, aux, wsb, ub, lam, stb2, side),
                                  args.steps, args.warmup, side)
            sg = snap.stats_to_numpy(stb2, B)
            hvg = max_violation(batch, ub.cpu().numpy())
            okg = (sg["status"] == 0) & (hvg <= H_FEAS)
            out[label] = {"value": int(okg.sum()) / secg, "ms_per_step": secg * 1e3,
                          "plan_create_s": tune_s,
                          "launch_groups": planb.describe().strip().splitlines()}

        if name == "burgers_godunov":
            # the paper's constraint-count study on its Godunov regime: one,
            # five and ten flux steps (IC and mass rows are not part of this family)
            fsweep = []
            for k in (1, 5, 10):
                bk = synthgen.make(name, nt=k + 1)
                pk = snap.Plan.from_batch(bk)
                wk = pk.new_workspace()
                uhk = torch.from_numpy(bk.uhat).to(dev)
                uk_ = torch.empty(pk.total_vars, dtype=torch.float64, device=dev)
                lk_ = torch.empty(max(pk.total_rows, 1), dtype=torch.float64, device=dev)
                sk_ = torch.empty(len(bk) * 32, dtype=torch.uint8, device=dev)
                axk = torch.from_numpy(bk.aux).to(dev)
                seck = time_calls(lambda: snap.project(pk, uhk, axk, wk, uk_, lk_, sk_, stream),
                                  args.steps, args.warmup, stream)
                stk = snap.stats_to_numpy(sk_, len(bk))
                hvk = max_violation(bk, uk_.cpu().numpy())
                okk = int(((stk["status"] == 0) & (hvk <= H_FEAS)).sum())
                fsweep.append({"flux_steps": k, "rows_per_sample": bk.samples[0].m,
                               "ms_per_step": seck * 1e3, "projected": okk, "value": okk / seck})
            out["flux_steps_sweep"] = fsweep

        # the constrained flow-matching sampler around the projection: N
        # substeps of shoot -> project (plain FP64, one plan and workspace for
        # all) -> pull back, from a N(0, 1) prior draw towards a Gaussian of
        # spread 0.05 about the batch's u_hat
        nsub, calls = 4, 2
        planp = snap.Plan.from_batch(batch)
        u0 = torch.from_numpy(synthgen.prior_sample(batch, seed=11)).to(dev)
        snap.pcfm_sample(planp, u0, uhat, 0.05, nsub, aux, stream)
        torch.cuda.synchronize()
        ep0, ep1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ep0.record(stream)
        for _ in range(calls):
            _, _, okp = snap.pcfm_sample(planp, u0, uhat, 0.05, nsub, aux, stream)
        ep1.record(stream)
        torch.cuda.synchronize()
        msp = ep0.elapsed_time(ep1) / calls
        out["pcfm"] = {"substeps": nsub, "ms_per_call": msp, "ms_per_substep": msp / nsub,
                       "converged_every_substep": int(okp[:B].sum().item())}

    if banded:
        # roofline of the dominant kernel, the banded factorization: the
        # method's flops (m b^2 per factorization, one per Newton step of
        # each sample) per launch over its average event-timed duration
        fms, flaunch, fdrop = plan64.kernel_times(snap.KERNEL_BAND_FACTOR)
        sms, slaunch, _ = plan64.kernel_times(snap.KERNEL_BAND_SOLVE)
        plan64.set_kernel_timing(False)
        flops, sbytes = band_work(batch, stats["newton_iters"])
        # every call launches max_newton factorizations per banded group
        # (converged samples return at once); marks past the timer's pool are
        # dropped, so scale the work to the launches actually timed
        n_band = sum(1 for l in plan64.describe().splitlines() if " band " in l)
        expected = args.steps * n_band * plan64.options.max_newton
        timed_frac = min(1.0, flaunch / max(expected, 1))
        per_launch = flops * args.steps * timed_frac / max(flaunch, 1)
        avg_s = fms / 1e3 / max(flaunch, 1)
        achieved = per_launch / avg_s / 1e12
        out["roofline"] = {
            "bound": "mfma", "achieved": achieved, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / FP64_PEAK_TFLOPS, "traffic": load_traffic(name),
            "kernel": KERNEL_NAMES[name], "flops_per_launch": per_launch,
            "avg_launch_ms": avg_s * 1e3, "launches_per_step": flaunch / args.steps,
            "dropped_marks": fdrop}
        s_per_launch = sbytes * args.steps * min(1.0, slaunch / max(expected, 1)) / max(slaunch, 1)
        s_avg = sms / 1e3 / max(slaunch, 1)
        out["roofline_band_solve"] = {
            "bound": "hbm", "achieved": s_per_launch / s_avg / 1e9, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": s_per_launch / s_avg / 1e9 / HBM_PEAK_GBS,
            "kernel": "band_solve", "bytes_per_launch": s_per_launch, "avg_launch_ms": s_avg * 1e3}
    elif name == "diff2d_energy":
        # one spectral-kernel launch per call: per Newton iteration a sample
        # must read u and u_hat and write u and lambda (float64)
        abytes = sum(max(int(it), 1) * 8 * (3 * s.n + s.m)
                     for s, it in zip(batch.samples, stats["newton_iters"]))
        lsec = launch_seconds(fwd64, args.steps, stream)
        achieved = abytes / lsec / 1e9
        out["roofline"] = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": achieved / HBM_PEAK_GBS, "traffic": load_traffic(name),
                           "kernel": KERNEL_NAMES[name], "algorithmic_bytes_per_launch": abytes,
                           "avg_launch_ms": lsec * 1e3}
    else:
        # roofline of the dominant kernel: the forward is one slab-kernel (or
        # boundary-row kernel) launch; events on the launch stream bracket it
        abytes = algorithmic_bytes(batch)
        lsec = launch_seconds(fwd64, args.steps, stream)
        achieved = abytes / lsec / 1e9
        out["roofline"] = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": achieved / HBM_PEAK_GBS, "traffic": load_traffic(name),
                           "kernel": KERNEL_NAMES[name], "algorithmic_bytes_per_launch": abytes,
                           "avg_launch_ms": lsec * 1e3}

    if cb is not None:
        out["cpu_baseline"] = cb
        errs = []
        for i, uo in orc.items():
            if uo is None:
                continue
            o, n = batch.var_off[i], batch.samples[i].n
            errs.append(np.linalg.norm(u_np[o:o + n] - uo) / max(np.linalg.norm(uo), 1e-300))
        out["parity"] = {"max_rel_u_vs_oracle": float(max(errs)), "samples": len(errs),
                         "oracle_not_converged": sum(1 for uo in orc.values() if uo is None)}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
