"""Batched constraint projection on MI355X (gfx950): Python binding.

Thin ctypes layer over the C ABI in include/snap.h (libsnap.so, built in-tree
by ``paper_2607_00095_amd.build``).  PyTorch supplies device memory and the
current stream only; every step of the projection runs in the HIP kernels.
The library must be built: importing this package without libsnap.so raises.

    plan = Plan(descs, options)                  # once per batch layout
    u, lam, stats = project(plan, uhat, aux)     # forward (u* and multipliers)
    g_uhat, _ = project_backward(plan, u, lam, aux, ws, grad_u)
    u = SnapProject.apply(uhat, aux, plan)       # autograd: d u*/d u_hat
"""
from .api import (  # noqa: F401
    BURGERS_BC, BURGERS_GODUNOV, BURGERS_LF, DIFF2D_ENERGY, FISHER_KPP, MASS_IC, PREC_FP64, PREC_MIXED, FLAG_KEEP_FACTOR,
    FLAG_GRAPH, FLAG_AUTOTUNE, FLAG_SOC, KERNEL_BAND_FACTOR, KERNEL_BAND_SOLVE,
    Options, Plan, SnapError, SnapProject, lib_path, pcfm_sample, project, project_backward,
    stats_to_numpy, status_name,
)
