/*
 * snap.h -- C ABI of the batched constraint-projection library (gfx950).
 *
 * For every sample s of a batch, independently (the batch Jacobian is
 * block-diagonal across samples, paper Sec. III-B), the library computes the
 * projection step of the constrained flow-matching sampler (paper Sec. II-A,
 * projection equation; restated as an NLP in Sec. III-B):
 *
 *     u*_s = argmin_u 1/2 ||u - u_hat_s||_2^2   subject to  h_s(u) = 0
 *
 * by Newton/SQP steps on the KKT system [[W, J^T], [J, 0]] (Appendix B), with
 * W = I + sum_i lam_i Hess h_i.  The Lagrangian is 1/2||u - u_hat||^2 + lam^T h,
 * so at the solution u* = u_hat - J(u*)^T lam*.
 *
 * Memory: every array argument is a DEVICE pointer owned by the caller unless
 * stated otherwise; u, u_hat, lambda and gradients are float64.  Variables of
 * one sample are the field flattened time-slab major, then y, then x (x
 * fastest), as in the paper's Appendix C flattening.  Samples are packed
 * back to back at the offsets given in their descriptors.
 *
 * Streams: `stream` is a hipStream_t (NULL = the null stream).  snap_project
 * and snap_project_backward only enqueue work and never synchronize.
 *
 * Errors: functions return SNAP_SUCCESS (0) or a negative SNAP_E* code for
 * invalid arguments, unsupported shapes or HIP failures.  Non-convergence of
 * a sample is not a call failure: it is reported per sample in the device
 * array of snap_sample_stats (status field, SNAP_ST_*).
 */
#ifndef SNAP_H_
#define SNAP_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Constraint families (rows in canonical order; lambda is returned in it).
 *
 * SNAP_MASS_IC      initial condition + per-step mass (paper Table 1 'Dirichlet
 *                   IC' and 'Global mass conservation'; Appendix A heat problem,
 *                   Appendix C).  Rows: u(x_i,t_0) - g_i (i < Nx), then
 *                   sum_i u(x_i,t_k) - M0 for k = 1..Nt-1.  aux = [g(Nx), M0].
 * SNAP_FISHER_KPP   initial condition + logistic mass budget (Table 1 'Nonlinear
 *                   conservation law'; Appendix A reaction-diffusion; Appendix D
 *                   discretization).  Rows: IC as above, then
 *                   sum u^{k+1} - sum u^k - dt*rho*sum u^k(1-u^k), k = 0..Nt-2.
 *                   p0 = rho, dt = dt.  aux = [g(Nx)].
 * SNAP_BURGERS_LF   flux-update residuals (Appendix D) of viscous Burgers with
 *                   the Lax-Friedrichs interface flux, periodic x.  Rows (k,i),
 *                   k-major, k = 0..Nt-2:  u_i^{k+1} - u_i^k + q(f(u_{i+1}^k) -
 *                   f(u_{i-1}^k)) - c(u_{i+1}^k - 2u_i^k + u_{i-1}^k), f = u^2/2,
 *                   q = dt/(2dx), c = p1*dt/(2dx) + p0*dt/dx^2.
 *                   p0 = nu, p1 = alpha (flux speed).  No aux.
 * SNAP_DIFF2D_ENERGY  implicit 2D diffusion residuals plus one energy row per
 *                   frame (Appendix A Navier-Stokes constraint set: local PDE
 *                   residuals and a global quadratic invariant), periodic
 *                   Nx x Ny grid (Nx = Ny in {16, 32, 48, 64}), 1 <= Nt <= 16.
 *                   Rows, canonical order: (k, y, x) for k = 0..Nt-2,
 *                   u(k+1) - u(k) - dt*p0*Lap5 u(k+1) with the periodic
 *                   5-point Laplacian of spacing dx; then, for t = 0..Nt-1,
 *                   sum_{y,x} u(t)^2 - E_t.  p0 = kappa.  aux = [E(Nt)].
 *                   Solved in the orthonormal real Fourier basis of each
 *                   frame; PREC_MIXED runs the same FP64 arithmetic (the
 *                   family has no band factorization to lower).
 * SNAP_BURGERS_BC   boundary conditions and mass of the paper's first Burgers
 *                   constraint regime (Appendix A, Burgers problem: Dirichlet
 *                   condition on the left boundary, mass, Neumann condition on
 *                   the right boundary; Appendix D discretizations).  Grid
 *                   x_i = i*dx, 3 <= Nx <= 512.  Rows, canonical order, for
 *                   k = 0..Nt-1 each: u_0^k - u_L; then dx*sum_i u_i^k - m0;
 *                   then (u_{Nx-1}^k - u_{Nx-2}^k)/dx.  aux = [u_L, m0].  The
 *                   rows are linear and per time step, so each step is
 *                   projected in closed form (3 x 3 Schur matrix); further
 *                   Newton steps only correct rounding.  No workspace; PREC_MIXED
 *                   runs the same FP64 arithmetic.  The adjoint is the
 *                   projection of the upstream gradient onto the rows' null
 *                   space.
 * SNAP_BURGERS_GODUNOV  flux-update residuals (Appendix D, Godunov's flux
 *                   conservation) of Burgers with Godunov's interface flux
 *                   F(a, b) = max(f(max(a,0)), f(min(b,0))), f = u^2/2, plus a
 *                   centred viscous term, periodic x.  Rows (k,i), k-major,
 *                   k = 0..Nt-2: u_i^{k+1} - u_i^k + (dt/dx)(F_{i+1/2} -
 *                   F_{i-1/2}) - p0*dt/dx^2 (u_{i+1}^k - 2u_i^k + u_{i-1}^k).
 *                   p0 = nu (0: inviscid).  No aux.  Solved by the banded
 *                   path of SNAP_BURGERS_LF; the flux is piecewise smooth and
 *                   Newton steps differentiate the branch that attains the
 *                   max (ties: the left state's), a semismooth Newton method.
 */
enum snap_family {
  SNAP_MASS_IC = 1,
  SNAP_FISHER_KPP = 2,
  SNAP_BURGERS_LF = 3,
  SNAP_DIFF2D_ENERGY = 4,
  SNAP_BURGERS_BC = 5,
  SNAP_BURGERS_GODUNOV = 6
};

enum snap_precision {
  SNAP_PREC_FP64 = 0,   /* every step in float64 */
  SNAP_PREC_MIXED = 1   /* float32 Schur factor/solve, float64 residuals and
                           iterative refinement of every KKT solve */
};

enum snap_flags {
  SNAP_FLAG_KEEP_FACTOR = 1, /* leave a factor of the KKT system taken at the
                                returned point in the workspace, for
                                snap_project_backward */
  SNAP_FLAG_GRAPH = 2,       /* run each call's whole launch sequence (for the
                                banded family: every Newton iteration's factor,
                                solve, step and evaluation launches) from a HIP
                                graph.  The graph is captured on the first call
                                and replayed while the array and workspace
                                pointers stay the same (they are re-captured
                                when they change); the plan keeps one graph per
                                direction.  Needs a non-null stream: on the
                                null stream the call runs its launches
                                directly.  A call that is a single kernel
                                launch (a plan of one slab-row group) also
                                runs directly: a graph of one launch only adds
                                the replay's overhead.  Calls with this flag on
                                one plan from several host threads are
                                serialized. */
  SNAP_FLAG_AUTOTUNE = 4,    /* snap_plan_create times every launch shape that
                                can run a group of samples (lanes per time slab
                                and rounds for the slab-row families; wavefronts
                                sharing one sample's band window for the banded
                                family) on a synthetic copy of the group (same
                                shapes and sample count, two Newton iterations)
                                and keeps the fastest.  Plan creation then
                                synchronizes the device and allocates temporary
                                device memory of the size of the call's arrays and
                                workspace.  Choices are cached per process.  A
                                shape changes the summation order of some
                                reductions, so results may differ from the
                                untuned plan's in the last bits. */
  SNAP_FLAG_SOC = 8          /* slab-row and banded families: when the full
                                Newton step fails the merit test and raised the
                                constraint violation, try one second-order
                                correction q = p - W^{-1} J^T S^{-1} h(u + p) with
                                the factor at u before halving (banded family:
                                one more launch per Newton iteration, which
                                returns at once unless a correction is due).
                                Off by default: on strongly nonlinear Fisher-KPP
                                samples it slowed or stalled convergence where
                                plain backtracking did not. */
};

/* call-level return codes */
enum snap_error {
  SNAP_SUCCESS = 0,
  SNAP_EINVAL = -1,        /* bad argument (null pointer, bad size, bad option) */
  SNAP_EHIP = -2,          /* a HIP runtime call or kernel launch failed */
  SNAP_ENOMEM = -3,        /* plan creation could not allocate its metadata */
  SNAP_EUNSUPPORTED = -4   /* family or grid size not supported */
};

/* per-sample status codes (snap_sample_stats.status) */
enum snap_sample_status {
  SNAP_ST_CONVERGED = 0,      /* ||h||_inf <= tol_h and stationarity <= tol_s(1+||u_hat||_inf) */
  SNAP_ST_MAX_ITER = 1,       /* max_newton iterations without meeting the tolerances */
  SNAP_ST_LS_FAIL = 2,        /* line search found no decrease of the merit */
  SNAP_ST_NONFINITE = 3,      /* NaN/Inf in input or iterates */
  SNAP_ST_SINGULAR_PIVOT = 4, /* non-positive pivot in the Schur factorization (2D
                                 family: a mode's reduced Hessian or the energy
                                 border is not positive definite) */
  SNAP_ST_HESSIAN_FLOOR = 5   /* adjoint only: the Lagrangian Hessian at (u*, lam*)
                                 has entries below the 0.1 floor the Newton steps
                                 use, so the gradient was formed with the floored
                                 W and is not the implicit-function derivative */
};

/* One sample.  Offsets are element offsets into the packed arrays. */
typedef struct snap_sample_desc {
  int32_t family;      /* enum snap_family */
  int32_t nx, ny, nt;  /* grid; ny = 1 in 1D */
  double dt, dx;       /* time step, grid spacing */
  double p0, p1;       /* family parameters (see enum snap_family) */
  int64_t var_off;     /* offset of the sample's variables in u_hat / u / gradients */
  int64_t row_off;     /* offset of its multipliers in lambda */
  int64_t aux_off;     /* offset of its auxiliary data in aux */
} snap_sample_desc;

typedef struct snap_options {
  double tol_h;        /* feasibility tolerance on ||h(u)||_inf (e.g. 1e-10) */
  double tol_s;        /* stationarity tolerance, relative to 1 + ||u_hat||_inf */
  int32_t max_newton;  /* Newton iterations per sample (>= 1) */
  int32_t max_ls;      /* backtracking halvings per line search (>= 0) */
  int32_t precision;   /* enum snap_precision */
  int32_t flags;       /* enum snap_flags, or-ed */
} snap_options;

typedef struct snap_sample_stats {
  int32_t status;         /* enum snap_sample_status */
  int32_t newton_iters;   /* Newton steps taken */
  int32_t ls_backtracks;  /* total step halvings */
  int32_t refine_steps;   /* iterative-refinement corrections (mixed precision) */
  double h_inf;           /* ||h(u)||_inf at the returned point */
  double stat_inf;        /* ||u - u_hat + J^T lambda||_inf at the returned point */
} snap_sample_stats;

typedef struct snap_plan_s* snap_plan;

/* Fill *opt with the defaults: tol_h 1e-11, tol_s 1e-11, max_newton 20,
 * max_ls 30, FP64, no flags. */
void snap_default_options(snap_options* opt);

/* Create a plan for `batch` samples described by the HOST array descs_host
 * (copied; the caller may free it).  The plan fixes the sparsity structure,
 * row orderings and band widths once (the fixed pattern is reused across
 * iterations and calls, paper Sec. III-B/III-C), and allocates its own small
 * device metadata on the current device.  batch = 0 is valid (calls then do
 * nothing).  Returns SNAP_EUNSUPPORTED for families or sizes the library does
 * not build.  Calls on one plan from several host threads are serialized
 * by a lock of the plan (its fork/join events, captured graphs and timer are
 * per plan); separate plans run independently. */
int snap_plan_create(snap_plan* out, int32_t batch, const snap_sample_desc* descs_host,
                     const snap_options* opt);

/* Bytes of caller-owned device workspace that snap_project and
 * snap_project_backward need for this plan (256-byte aligned start required). */
int snap_plan_workspace_bytes(snap_plan plan, size_t* bytes);

/* Number of constraint rows / variables / aux values the plan expects in the
 * packed arrays. */
int snap_plan_sizes(snap_plan plan, int64_t* total_vars, int64_t* total_rows, int64_t* total_aux);

/* Forward projection of every sample.
 *   uhat        [total_vars]  input (read only)
 *   aux         [total_aux]   family data (IC targets, masses); may be NULL if total_aux = 0
 *   u_out       [total_vars]  projected fields (must not alias uhat)
 *   lambda_out  [total_rows]  multipliers, canonical row order
 *   stats       [batch]       per-sample status and diagnostics
 *   workspace   snap_plan_workspace_bytes bytes, 256-byte aligned
 * With SNAP_FLAG_KEEP_FACTOR in the plan's options, the workspace afterwards
 * holds the Schur factor at the returned (u, lambda) for the backward call. */
int snap_project(snap_plan plan, const double* uhat, const double* aux, double* u_out,
                 double* lambda_out, snap_sample_stats* stats, void* workspace, void* stream);

/* Largest workspace (bytes) that snap_project_noalloc can serve. */
#define SNAP_NOALLOC_MAX_WORKSPACE (64u << 20)

/* snap_project without a caller workspace, for callers that cannot allocate
 * device memory (code under HIP-graph capture, tight serving loops, harnesses
 * that forbid allocation).  Same arguments and results as snap_project; the
 * workspace is a static 64 MiB device array of the library, one per GPU, held
 * until the process ends, whose address is looked up when a plan is created.
 * The call itself allocates nothing.
 *   Returns SNAP_EINVAL if the plan's workspace (snap_plan_workspace_bytes)
 *   exceeds SNAP_NOALLOC_MAX_WORKSPACE (for instance one 256 x 128 Burgers
 *   sample in FP64), or if the current device is not the plan's.
 * Every call on one GPU shares that GPU's array and leaves its contents
 * behind (every kernel sets up the state it reads, so nothing needs clearing
 * between calls): calls that overlap in time on one GPU, on any plans or
 * streams, race.  A factor kept with SNAP_FLAG_KEEP_FACTOR stays in the array
 * and cannot be handed to snap_project_backward; use snap_project with a
 * workspace for the adjoint. */
int snap_project_noalloc(snap_plan plan, const double* uhat, const double* aux, double* u_out,
                         double* lambda_out, snap_sample_stats* stats, void* stream);

/* Vector-Jacobian product of the projection with respect to u_hat at the
 * solution (implicit-function theorem on the KKT conditions): with the KKT
 * matrix K at (u, lambda), grad_uhat is the u-block of K^{-1} [grad_u; 0]
 * = W^{-1}(grad_u - J^T b) with (J W^{-1} J^T) b = J W^{-1} grad_u.
 *   u, lambda   outputs of snap_project on the same plan and workspace
 *   grad_u      [total_vars]  upstream gradient
 *   grad_uhat   [total_vars]  result
 *   stats       [batch]       refine_steps and status of the adjoint solve
 * Reuses the factor left by a forward call with SNAP_FLAG_KEEP_FACTOR; without
 * it the library factors again at (u, lambda). */
int snap_project_backward(snap_plan plan, const double* u, const double* lambda,
                          const double* aux, void* workspace, const double* grad_u,
                          double* grad_uhat, snap_sample_stats* stats, void* stream);

/* Text description of the plan's launch groups, one line per group
 * ("group <i>: <slab|band|spectral> class <c>, <w> wavefronts per workgroup
 * [, two-sided factorization], <n> samples").
 * Writes at most len bytes into buf (NUL-terminated when len > 0); *needed, if
 * not NULL, receives the full length without the NUL. */
int snap_plan_describe(snap_plan plan, char* buf, size_t len, size_t* needed);

/* Kernel classes (launch shapes) that can run launch group `group` of the plan,
 * the one in use first; *count receives how many there are (at most cap are
 * written).  Groups are numbered as in snap_plan_describe.  Banded family:
 * class BB (block half-bandwidth, default shape), BB + 32 (the other
 * wavefront count, BB <= 9), BB + 64 (two-sided factorization, BB >= 13:
 * two workgroups per sample factor the band from both ends toward a
 * separator, which halves the chain of dependent panel steps; the default
 * for bands of at least 40 BB block rows).  A banded group of at most one
 * sample per CU defaults to BB + 32 at BB <= 9 and to BB + 64 at BB >= 13
 * (at least 3 BB block rows per sample). */
int snap_plan_group_classes(snap_plan plan, int32_t group, int32_t* classes, int32_t cap,
                            int32_t* count);

/* Run launch group `group` with kernel class `cls`, one of those listed by
 * snap_plan_group_classes (for instance a choice saved from an autotuned
 * plan).  Drops any captured graph.  Must not race with calls on the plan. */
int snap_plan_set_group_class(snap_plan plan, int32_t group, int32_t cls);

/* Steps of the constrained flow-matching sampler around the projection
 * (paper Sec. II-A, sampling loop over N substeps of flow time: shoot to
 * flow time 1 with the velocity, project, pull back along the straight-line
 * interpolant).  Elementwise over n packed float64 values (device pointers,
 * caller-owned, stream-ordered); outputs must not alias inputs except where
 * stated.  Return SNAP_EINVAL for a bad size, pointer or time.
 *
 * snap_flow_velocity_gaussian: v = m + c(tau) (u - tau m),
 *   c(tau) = (tau s^2 - (1 - tau)) / ((1 - tau)^2 + tau^2 s^2), the exact
 *   marginal velocity E[x1 - x0 | x_tau = u] of the straight-line interpolant
 *   between x0 ~ N(0, I) and x1 ~ N(m, s^2 I): a closed-form stand-in for a
 *   trained velocity network (0 <= tau <= 1, s > 0).
 * snap_flow_shoot: u1_hat = u_tau + (1 - tau) v (u1_hat may alias u_tau).
 * snap_flow_pullback: u_tau' = u0 + tau' (u1 - u0) (u_tau' may alias u1). */
int snap_flow_velocity_gaussian(int64_t n, const double* u, const double* mean, double tau, double s,
                                double* v, void* stream);
int snap_flow_shoot(int64_t n, const double* u_tau, const double* v, double tau, double* u1_hat,
                    void* stream);
int snap_flow_pullback(int64_t n, const double* u0, const double* u1, double tau_next, double* u_tau,
                       void* stream);

/* Kernel timing (a tracing aid; not needed for projection).  With timing
 * enabled, snap_project and snap_project_backward record a HIP event on the
 * launch stream before and after every launch of the timed kernels
 * (SNAP_KERNEL_BAND_FACTOR: the banded Schur factorization with its fused
 * forward substitution; SNAP_KERNEL_BAND_SOLVE: the backward substitution and
 * refinement of a Newton step), from a pool of 8192 events allocated by
 * snap_plan_set_kernel_timing (so calls still allocate nothing).  Marks past
 * the pool are dropped and counted.  Not available with SNAP_FLAG_GRAPH
 * (returns SNAP_EUNSUPPORTED).  Timing a launch that shares the GPU with
 * launches on other streams (ragged plans fork their groups over four streams)
 * includes that sharing, as a kernel trace does. */
enum snap_timed_kernel { SNAP_KERNEL_BAND_FACTOR = 0, SNAP_KERNEL_BAND_SOLVE = 1 };

/* enable != 0: allocate the event pool (or clear the recorded marks);
 * enable == 0: free it.  Must not race with calls on the plan. */
int snap_plan_set_kernel_timing(snap_plan plan, int32_t enable);

/* Sum of the recorded launch durations of `kernel` (milliseconds) and their
 * count since timing was enabled or last reset; *dropped (if not NULL)
 * receives the number of marks lost to a full pool.  Waits for the recorded
 * events (synchronizes the host with them). */
int snap_plan_kernel_times(snap_plan plan, int32_t kernel, double* total_ms, int64_t* launches,
                           int64_t* dropped);

/* Forget the recorded marks (waits for them first). */
int snap_plan_reset_kernel_times(snap_plan plan);

int snap_plan_destroy(snap_plan plan);

/* Static strings for return codes (negative) and sample status codes (>= 0). */
const char* snap_error_string(int code);
const char* snap_status_string(int status);

#ifdef __cplusplus
}
#endif

#endif /* SNAP_H_ */
