// Elementwise steps of the constrained flow-matching sampler around the
// projection (paper Sec. II-A, sampling loop): the one-step shoot to flow
// time 1, the straight-line pull-back, and a closed-form velocity (the exact
// marginal velocity of a Gaussian target) standing in for a trained network.
// Streaming kernels: one read of each input and one write per element,
// consecutive lanes on consecutive elements, grid-stride over the batch.
#include "snap_device.hpp"

namespace snap {

namespace {

constexpr int kFlowThreads = 256;

__global__ __launch_bounds__(kFlowThreads) void flow_velocity_kernel(int64_t n, const double* u,
                                                                     const double* mean, double tau,
                                                                     double c, double* v) {
  const int64_t stride = (int64_t)gridDim.x * kFlowThreads;
  for (int64_t i = (int64_t)blockIdx.x * kFlowThreads + threadIdx.x; i < n; i += stride) {
    const double m = mean[i];
    v[i] = m + c * (u[i] - tau * m);
  }
}

__global__ __launch_bounds__(kFlowThreads) void flow_shoot_kernel(int64_t n, const double* u,
                                                                  const double* v, double rem,
                                                                  double* out) {
  const int64_t stride = (int64_t)gridDim.x * kFlowThreads;
  for (int64_t i = (int64_t)blockIdx.x * kFlowThreads + threadIdx.x; i < n; i += stride)
    out[i] = u[i] + rem * v[i];
}

__global__ __launch_bounds__(kFlowThreads) void flow_pullback_kernel(int64_t n, const double* u0,
                                                                     const double* u1, double tn,
                                                                     double* out) {
  const int64_t stride = (int64_t)gridDim.x * kFlowThreads;
  for (int64_t i = (int64_t)blockIdx.x * kFlowThreads + threadIdx.x; i < n; i += stride) {
    const double a = u0[i];
    out[i] = a + tn * (u1[i] - a);
  }
}

dim3 flow_grid(int64_t n) {
  // enough workgroups to fill every CU several times over; grid-stride beyond
  const int64_t g = (n + kFlowThreads - 1) / kFlowThreads;
  return dim3((unsigned)(g < 8192 ? (g > 0 ? g : 1) : 8192));
}

}  // namespace

}  // namespace snap

using namespace snap;

extern "C" {

int snap_flow_velocity_gaussian(int64_t n, const double* u, const double* mean, double tau, double s,
                                double* v, void* stream) {
  if (n < 0 || (n > 0 && (!u || !mean || !v)) || !(tau >= 0.0 && tau <= 1.0) || !(s > 0.0))
    return SNAP_EINVAL;
  if (n == 0) return SNAP_SUCCESS;
  const double var = (1.0 - tau) * (1.0 - tau) + tau * tau * s * s;
  const double c = (tau * s * s - (1.0 - tau)) / var;
  hipLaunchKernelGGL(flow_velocity_kernel, flow_grid(n), dim3(kFlowThreads), 0, (hipStream_t)stream,
                     n, u, mean, tau, c, v);
  return hipGetLastError() == hipSuccess ? SNAP_SUCCESS : SNAP_EHIP;
}

int snap_flow_shoot(int64_t n, const double* u_tau, const double* v, double tau, double* u1_hat,
                    void* stream) {
  if (n < 0 || (n > 0 && (!u_tau || !v || !u1_hat)) || !(tau >= 0.0 && tau <= 1.0)) return SNAP_EINVAL;
  if (n == 0) return SNAP_SUCCESS;
  hipLaunchKernelGGL(flow_shoot_kernel, flow_grid(n), dim3(kFlowThreads), 0, (hipStream_t)stream,
                     n, u_tau, v, 1.0 - tau, u1_hat);
  return hipGetLastError() == hipSuccess ? SNAP_SUCCESS : SNAP_EHIP;
}

int snap_flow_pullback(int64_t n, const double* u0, const double* u1, double tau_next, double* u_tau,
                       void* stream) {
  if (n < 0 || (n > 0 && (!u0 || !u1 || !u_tau)) || !(tau_next >= 0.0 && tau_next <= 1.0))
    return SNAP_EINVAL;
  if (n == 0) return SNAP_SUCCESS;
  hipLaunchKernelGGL(flow_pullback_kernel, flow_grid(n), dim3(kFlowThreads), 0, (hipStream_t)stream,
                     n, u0, u1, tau_next, u_tau);
  return hipGetLastError() == hipSuccess ? SNAP_SUCCESS : SNAP_EHIP;
}

}  // extern "C"
