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
};

__device__ __forceinline__ double bcast_first(double v) {
  int lo = __builtin_amdgcn_readfirstlane(__double2loint(v));
  int hi = __builtin_amdgcn_readfirstlane(__double2hiint(v));
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ float bcast_first(float v) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}

// Butterfly sum over the 64 lanes; the result of lane 0 is broadcast so every
// lane holds bit-identical values.
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return bcast_first(v);
}

template <typename T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, kWave));
  return bcast_first(v);
}

__device__ __forceinline__ bool finite(double v) { return __builtin_isfinite(v); }

// Order LDS accesses of one wavefront (no cross-wave synchronization).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

}  // namespace snap
