// Device-side helpers shared by the gfx950 kernels of the projection library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "snap.h"

namespace snap {

constexpr int kWave = 64;

// Launch arguments common to every family kernel.
struct KernelArgs {
  const snap_sample_desc* descs;   // device copy of the plan's descriptors
  const int32_t* order;            // sample ids processed by this launch
  int32_t count;                   // number of entries in `order`
  const double* uhat;
  const double* aux;
  double* u;                       // forward: output field; backward: u* (read only)
  double* lam;                     // forward: output multipliers; backward: lambda* (read only)
  snap_sample_stats* stats;
  const double* grad_u;            // backward only
  double* grad_uhat;               // backward only
  unsigned char* ws;               // workspace base
  const int64_t* ws_off;           // per-sample byte offset of its workspace block (or null)
  snap_options opt;
  int32_t backward;                // 0 = forward projection, 1 = adjoint
  const double* tab;               // Fourier basis tables of the 2D family (or null)
};

__device__ __forceinline__ double bcast_first(double v) {
  int lo = __builtin_amdgcn_readfirstlane(__double2loint(v));
  int hi = __builtin_amdgcn_readfirstlane(__double2hiint(v));
  return __hiloint2double(hi, lo);
}

// Wavefront reductions with DPP (VALU only, no LDS round trips): an
// inclusive prefix within each row of 16 lanes (row_shr 1, 2, 4, 8), then
// row_bcast:15 / row_bcast:31 fold rows together, so lane 63 holds the
// result; it is broadcast so every lane holds bit-identical values.
// Out-of-row sources read 0 (bound_ctrl): valid for sums and for maxima of
// non-negative values, which is how these are used.
template <int CTRL, int ROWMASK, bool BC>
__device__ __forceinline__ double dpp_d(double x) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), CTRL, ROWMASK, 0xf, BC);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), CTRL, ROWMASK, 0xf, BC);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double lane63(double v) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_d<0x111, 0xf, true>(v);    // row_shr:1
  v += dpp_d<0x112, 0xf, true>(v);    // row_shr:2
  v += dpp_d<0x114, 0xf, true>(v);    // row_shr:4
  v += dpp_d<0x118, 0xf, true>(v);    // row_shr:8
  v += dpp_d<0x142, 0xa, false>(v);   // row_bcast:15 into rows 1, 3
  v += dpp_d<0x143, 0xc, false>(v);   // row_bcast:31 into rows 2, 3
  return lane63(v);
}

// maximum of non-negative values
__device__ __forceinline__ double wave_max(double v) {
  v = fmax(v, dpp_d<0x111, 0xf, true>(v));
  v = fmax(v, dpp_d<0x112, 0xf, true>(v));
  v = fmax(v, dpp_d<0x114, 0xf, true>(v));
  v = fmax(v, dpp_d<0x118, 0xf, true>(v));
  v = fmax(v, dpp_d<0x142, 0xa, false>(v));
  v = fmax(v, dpp_d<0x143, 0xc, false>(v));
  return lane63(v);
}

// Barriers that order LDS only: they do not wait for outstanding global
// loads or stores, so prefetches and factor write-back stay in flight.
// Global data exchanged between wavefronts still needs __syncthreads().
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

__device__ __forceinline__ bool finite(double v) { return __builtin_isfinite(v); }

// 1/b from the hardware estimate refined by Newton-Raphson steps
// (x <- x + x(1 - b x)), within about an ulp of the rounded quotient for
// normal, finite b; a few FMAs instead of the IEEE division sequence.
__device__ __forceinline__ double rcp_nr(double b) {
  double x = __builtin_amdgcn_rcp(b);
  double e = __builtin_fma(-b, x, 1.0);
  x = __builtin_fma(x, e, x);
  e = __builtin_fma(-b, x, 1.0);
  return __builtin_fma(x, e, x);
}
__device__ __forceinline__ float rcp_nr(float b) {
  const float x = __builtin_amdgcn_rcpf(b);
  const float e = __builtin_fmaf(-b, x, 1.0f);
  return __builtin_fmaf(x, e, x);
}

// Order LDS accesses of one wavefront (no cross-wave synchronization).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
}

// Optional per-kernel timing of a call's launch sequence
// (snap_plan_set_kernel_timing).  While a plan with timing enabled runs,
// `tl_timer` points at its timer and the launch code brackets the timed
// kernels with timer_mark(kernel, begin/end, stream), which records one event
// of a preallocated pool on the launch stream.  Host code only.
enum TimedKernel { kTimedBandFactor = 0, kTimedBandSolve = 1, kTimedCount = 2 };
struct KernelTimer;
extern thread_local KernelTimer* tl_timer;
void timer_mark(KernelTimer* t, int kernel, hipStream_t st);

}  // namespace snap
