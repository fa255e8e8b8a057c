"""ctypes marshalling for libsnap.so (argument conversion only)."""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np
import torch

MASS_IC, FISHER_KPP, BURGERS_LF, DIFF2D_ENERGY, BURGERS_BC, BURGERS_GODUNOV = 1, 2, 3, 4, 5, 6
PREC_FP64, PREC_MIXED = 0, 1
FLAG_KEEP_FACTOR, FLAG_GRAPH, FLAG_AUTOTUNE, FLAG_SOC = 1, 2, 4, 8
KERNEL_BAND_FACTOR, KERNEL_BAND_SOLVE = 0, 1

_HERE = os.path.dirname(os.path.abspath(__file__))


def lib_path() -> str:
    return os.path.join(_HERE, "libsnap.so")


class SnapError(RuntimeError):
    pass


class _Desc(C.Structure):
    _fields_ = [("family", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32), ("nt", C.c_int32),
                ("dt", C.c_double), ("dx", C.c_double), ("p0", C.c_double), ("p1", C.c_double),
                ("var_off", C.c_int64), ("row_off", C.c_int64), ("aux_off", C.c_int64)]


class _Opt(C.Structure):
    _fields_ = [("tol_h", C.c_double), ("tol_s", C.c_double), ("max_newton", C.c_int32),
                ("max_ls", C.c_int32), ("precision", C.c_int32), ("flags", C.c_int32)]


STATS_DTYPE = np.dtype([("status", "<i4"), ("newton_iters", "<i4"), ("ls_backtracks", "<i4"),
                        ("refine_steps", "<i4"), ("h_inf", "<f8"), ("stat_inf", "<f8")])

_STATUS = {0: "converged", 1: "max_iter", 2: "line_search_failed", 3: "nonfinite",
           4: "singular_pivot", 5: "hessian_floor"}


def status_name(code: int) -> str:
    return _STATUS.get(int(code), "unknown")


_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    path = lib_path()
    if not os.path.exists(path):
        raise SnapError(f"{path} is missing: build it with `python -m paper_2607_00095_amd.build` "
                        "(there is no CPU fallback)")
    lib = C.CDLL(path)
    vp, i32, i64, dp = C.c_void_p, C.c_int32, C.c_int64, C.POINTER(C.c_double)
    lib.snap_default_options.argtypes = [C.POINTER(_Opt)]
    lib.snap_default_options.restype = None
    lib.snap_plan_create.argtypes = [C.POINTER(vp), i32, C.POINTER(_Desc), C.POINTER(_Opt)]
    lib.snap_plan_workspace_bytes.argtypes = [vp, C.POINTER(C.c_size_t)]
    lib.snap_plan_sizes.argtypes = [vp, C.POINTER(i64), C.POINTER(i64), C.POINTER(i64)]
    lib.snap_project.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp]
    lib.snap_project_backward.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp]
    lib.snap_plan_destroy.argtypes = [vp]
    lib.snap_plan_describe.argtypes = [vp, C.c_char_p, C.c_size_t, C.POINTER(C.c_size_t)]
    lib.snap_plan_group_classes.argtypes = [vp, i32, C.POINTER(i32), i32, C.POINTER(i32)]
    lib.snap_plan_set_group_class.argtypes = [vp, i32, i32]
    lib.snap_plan_set_kernel_timing.argtypes = [vp, i32]
    lib.snap_plan_kernel_times.argtypes = [vp, i32, dp, C.POINTER(i64), C.POINTER(i64)]
    lib.snap_plan_reset_kernel_times.argtypes = [vp]
    lib.snap_flow_velocity_gaussian.argtypes = [i64, vp, vp, C.c_double, C.c_double, vp, vp]
    lib.snap_flow_shoot.argtypes = [i64, vp, vp, C.c_double, vp, vp]
    lib.snap_flow_pullback.argtypes = [i64, vp, vp, C.c_double, vp, vp]
    lib.snap_project_noalloc.argtypes = [vp] * 7
    lib.snap_error_string.argtypes = [C.c_int]
    lib.snap_error_string.restype = C.c_char_p
    lib.snap_status_string.argtypes = [C.c_int]
    lib.snap_status_string.restype = C.c_char_p
    for f in ("snap_plan_create", "snap_plan_workspace_bytes", "snap_plan_sizes", "snap_project",
              "snap_project_backward", "snap_plan_destroy", "snap_plan_describe",
              "snap_plan_group_classes", "snap_plan_set_group_class", "snap_plan_set_kernel_timing",
              "snap_plan_kernel_times", "snap_plan_reset_kernel_times", "snap_flow_velocity_gaussian",
              "snap_flow_shoot", "snap_flow_pullback", "snap_project_noalloc"):
        getattr(lib, f).restype = C.c_int
    _lib = lib
    return lib


def _check(rc: int, what: str):
    if rc != 0:
        msg = _load().snap_error_string(rc).decode()
        raise SnapError(f"{what} failed: {msg} ({rc})")


@dataclass
class Options:
    tol_h: float = 1e-11
    tol_s: float = 1e-11
    max_newton: int = 20
    max_ls: int = 30
    precision: int = PREC_FP64
    flags: int = 0

    def to_c(self) -> _Opt:
        return _Opt(self.tol_h, self.tol_s, self.max_newton, self.max_ls, self.precision, self.flags)


def descs_from_samples(samples, var_off, row_off, aux_off) -> Sequence[_Desc]:
    """Descriptors from objects with family/nx/ny/nt/dt/dx/p0/p1 attributes."""
    arr = (_Desc * len(samples))()
    for i, s in enumerate(samples):
        arr[i] = _Desc(int(s.family), int(s.nx), int(s.ny), int(s.nt), float(s.dt), float(s.dx),
                       float(s.p0), float(s.p1), int(var_off[i]), int(row_off[i]), int(aux_off[i]))
    return arr


class Plan:
    """Owns a snap_plan (fixed shapes, orderings, workspace layout)."""

    def __init__(self, samples, var_off, row_off, aux_off, options: Optional[Options] = None,
                 device=None):
        lib = _load()
        self.options = options or Options()
        self.batch = len(samples)
        self._descs = descs_from_samples(samples, var_off, row_off, aux_off)
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        h = C.c_void_p()
        opt = self.options.to_c()
        with torch.cuda.device(self.device):
            _check(lib.snap_plan_create(C.byref(h), self.batch, self._descs, C.byref(opt)),
                   "snap_plan_create")
        self._h = h
        nb = C.c_size_t()
        _check(lib.snap_plan_workspace_bytes(h, C.byref(nb)), "snap_plan_workspace_bytes")
        self.workspace_bytes = int(nb.value)
        tv, tr, ta = C.c_int64(), C.c_int64(), C.c_int64()
        _check(lib.snap_plan_sizes(h, C.byref(tv), C.byref(tr), C.byref(ta)), "snap_plan_sizes")
        self.total_vars, self.total_rows, self.total_aux = int(tv.value), int(tr.value), int(ta.value)

    @classmethod
    def from_batch(cls, batch, options: Optional[Options] = None, device=None):
        return cls(batch.samples, batch.var_off, batch.row_off, batch.aux_off, options, device)

    def describe(self) -> str:
        """One line per launch group: family kind, kernel class, wavefronts, samples."""
        lib = _load()
        need = C.c_size_t()
        _check(lib.snap_plan_describe(self._h, None, 0, C.byref(need)), "snap_plan_describe")
        buf = C.create_string_buffer(need.value + 1)
        _check(lib.snap_plan_describe(self._h, buf, need.value + 1, None), "snap_plan_describe")
        return buf.value.decode()

    def group_classes(self, group: int):
        """Kernel classes that can run launch group `group`, the one in use first."""
        lib = _load()
        arr = (C.c_int32 * 16)()
        n = C.c_int32()
        _check(lib.snap_plan_group_classes(self._h, group, arr, 16, C.byref(n)), "snap_plan_group_classes")
        return [arr[i] for i in range(min(n.value, 16))]

    def set_group_class(self, group: int, cls: int):
        _check(_load().snap_plan_set_group_class(self._h, group, cls), "snap_plan_set_group_class")

    def set_kernel_timing(self, enable: bool = True):
        _check(_load().snap_plan_set_kernel_timing(self._h, 1 if enable else 0),
               "snap_plan_set_kernel_timing")

    def kernel_times(self, kernel: int):
        """(total milliseconds, launches, dropped marks) of a timed kernel."""
        ms, n, dr = C.c_double(), C.c_int64(), C.c_int64()
        _check(_load().snap_plan_kernel_times(self._h, kernel, C.byref(ms), C.byref(n), C.byref(dr)),
               "snap_plan_kernel_times")
        return ms.value, n.value, dr.value

    def reset_kernel_times(self):
        _check(_load().snap_plan_reset_kernel_times(self._h), "snap_plan_reset_kernel_times")

    def new_workspace(self) -> torch.Tensor:
        # 256-byte aligned: torch's caching allocator returns 512-byte aligned blocks
        ws = torch.empty(max(self.workspace_bytes, 256), dtype=torch.uint8, device=self.device)
        assert ws.data_ptr() % 256 == 0
        return ws

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.snap_plan_destroy(h)
            self._h = None


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


def _dev_f64(t: torch.Tensor, n: int, name: str, device) -> torch.Tensor:
    if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise SnapError(f"{name} must be a contiguous float64 CUDA tensor")
    if t.numel() < n:
        raise SnapError(f"{name} has {t.numel()} elements, plan needs {n}")
    return t


def project(plan: Plan, uhat: torch.Tensor, aux: Optional[torch.Tensor],
            workspace: Optional[torch.Tensor] = None, u_out=None, lam_out=None, stats=None,
            stream: Optional[torch.cuda.Stream] = None):
    """Forward projection.  Returns (u, lam, stats_bytes, workspace)."""
    lib = _load()
    _dev_f64(uhat, plan.total_vars, "uhat", plan.device)
    if plan.total_aux > 0:
        _dev_f64(aux, plan.total_aux, "aux", plan.device)
    dev = plan.device
    u = u_out if u_out is not None else torch.empty(max(plan.total_vars, 1), dtype=torch.float64, device=dev)
    lam = lam_out if lam_out is not None else torch.empty(max(plan.total_rows, 1), dtype=torch.float64, device=dev)
    st = stats if stats is not None else torch.empty(max(plan.batch, 1) * STATS_DTYPE.itemsize,
                                                     dtype=torch.uint8, device=dev)
    ws = workspace if workspace is not None else plan.new_workspace()
    s = stream if stream is not None else torch.cuda.current_stream(dev)
    _check(lib.snap_project(plan._h, _ptr(uhat), _ptr(aux), _ptr(u), _ptr(lam), _ptr(st), _ptr(ws),
                            C.c_void_p(s.cuda_stream)), "snap_project")
    return u, lam, st, ws


def project_backward(plan: Plan, u: torch.Tensor, lam: torch.Tensor, aux: Optional[torch.Tensor],
                     workspace: torch.Tensor, grad_u: torch.Tensor, grad_out=None, stats=None,
                     stream: Optional[torch.cuda.Stream] = None):
    """Adjoint: returns (grad_uhat, stats_bytes)."""
    lib = _load()
    _dev_f64(grad_u, plan.total_vars, "grad_u", plan.device)
    dev = plan.device
    g = grad_out if grad_out is not None else torch.empty(max(plan.total_vars, 1), dtype=torch.float64, device=dev)
    st = stats if stats is not None else torch.empty(max(plan.batch, 1) * STATS_DTYPE.itemsize,
                                                     dtype=torch.uint8, device=dev)
    s = stream if stream is not None else torch.cuda.current_stream(dev)
    _check(lib.snap_project_backward(plan._h, _ptr(u), _ptr(lam), _ptr(aux), _ptr(workspace),
                                     _ptr(grad_u), _ptr(g), _ptr(st), C.c_void_p(s.cuda_stream)),
           "snap_project_backward")
    return g, st


def pcfm_sample(plan: Plan, u0: torch.Tensor, mean: torch.Tensor, s: float, nsteps: int,
                aux: Optional[torch.Tensor], stream: Optional[torch.cuda.Stream] = None):
    """Constrained flow-matching sampler (paper Sec. II-A) over `nsteps`
    uniform substeps of flow time, with the closed-form Gaussian velocity:
    shoot to flow time 1, project every sample with `plan`, pull back along
    the straight-line interpolant.  The plan and one workspace serve every
    substep.  Returns (sample, stats of the last projection, number of
    samples that converged in every substep)."""
    lib = _load()
    n = plan.total_vars
    _dev_f64(u0, n, "u0", plan.device)
    _dev_f64(mean, n, "mean", plan.device)
    if nsteps < 1:
        raise SnapError("nsteps must be >= 1")
    dev = plan.device
    st = stream if stream is not None else torch.cuda.current_stream(dev)
    sp = C.c_void_p(st.cuda_stream)
    u = u0.clone()
    v = torch.empty_like(u)
    u1 = torch.empty_like(u)
    lam = torch.empty(max(plan.total_rows, 1), dtype=torch.float64, device=dev)
    stats = torch.empty(max(plan.batch, 1) * STATS_DTYPE.itemsize, dtype=torch.uint8, device=dev)
    ok_all = torch.ones(max(plan.batch, 1), dtype=torch.bool, device=dev)
    ws = plan.new_workspace()
    for j in range(nsteps):
        tau, tau_next = j / nsteps, (j + 1) / nsteps
        _check(lib.snap_flow_velocity_gaussian(n, _ptr(u), _ptr(mean), tau, s, _ptr(v), sp),
               "snap_flow_velocity_gaussian")
        _check(lib.snap_flow_shoot(n, _ptr(u), _ptr(v), tau, _ptr(v), sp), "snap_flow_shoot")
        project(plan, v, aux, ws, u1, lam, stats, st)
        status = stats.view(torch.int32).view(-1, STATS_DTYPE.itemsize // 4)[: plan.batch, 0]
        ok_all &= status[: plan.batch] == 0
        if j + 1 < nsteps:
            _check(lib.snap_flow_pullback(n, _ptr(u0), _ptr(u1), tau_next, _ptr(u), sp),
                   "snap_flow_pullback")
    return u1, stats, ok_all


def stats_to_numpy(stats: torch.Tensor, batch: int) -> np.ndarray:
    raw = stats.detach().cpu().numpy()[: batch * STATS_DTYPE.itemsize]
    return raw.view(STATS_DTYPE)


class SnapProject(torch.autograd.Function):
    """u* = P(u_hat); backward gives the implicit-function VJP d u*/d u_hat.

    u_hat holds exactly plan.total_vars values (any shape); u* and the
    gradient have u_hat's shape.  The backward checks the forward's
    per-sample status (one device-to-host copy of the stats) and raises
    SnapError if a sample did not converge, since the implicit-function
    gradient only holds at a KKT point; pass allow_unconverged=True to get
    the gradient at the returned points anyway."""

    @staticmethod
    def forward(ctx, uhat, aux, plan: Plan, allow_unconverged: bool = False):
        if uhat.numel() != plan.total_vars:
            raise SnapError(f"u_hat has {uhat.numel()} values, the plan has {plan.total_vars}")
        u, lam, st, ws = project(plan, uhat.detach().contiguous().view(-1), aux)
        ctx.plan = plan
        ctx.shape = uhat.shape
        ctx.allow = allow_unconverged
        ctx.save_for_backward(u, lam, aux if aux is not None else torch.empty(0), ws, st)
        return u[: plan.total_vars].view(uhat.shape)

    @staticmethod
    def backward(ctx, grad_u):
        u, lam, aux, ws, st = ctx.saved_tensors
        plan = ctx.plan
        if not ctx.allow and plan.batch > 0:
            status = stats_to_numpy(st, plan.batch)["status"]
            if (status != 0).any():
                bad = np.flatnonzero(status != 0)
                raise SnapError(f"{bad.size} sample(s) did not converge in the forward "
                                f"(first: {bad[0]}, status {status_name(status[bad[0]])}); "
                                "their implicit-function gradient is undefined")
        g, _ = project_backward(plan, u, lam, aux if aux.numel() else None, ws,
                                grad_u.contiguous().view(-1).to(torch.float64))
        return g[: plan.total_vars].view(ctx.shape), None, None, None
