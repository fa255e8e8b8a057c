// Boundary rows and global mass of Burgers' first constraint regime (paper
// Appendix A, Burgers problem: Dirichlet condition on the left boundary,
// mass, Neumann condition on the right boundary; Appendix D discretizations:
// Riemann-sum mass, one-sided boundary difference).  Per time step k the rows
//   D_k = u_0 - u_L,   M_k = dx sum_x u_x - m0,   N_k = (u_{nx-1} - u_{nx-2}) / dx
// touch that step's slab only and are linear, so the projection is one
// Newton step per slab with the 3 x 3 Schur matrix S = A A^T in closed form
// (W = I: the Lagrangian Hessian of linear rows is the objective's):
//   S = [[1, dx, 0], [dx, nx dx^2, 0], [0, 0, 2 / dx^2]]   (nx >= 3)
// lam = S^{-1} (A u - b), u -= A^T lam.  A second step from the result (the
// same formulas on its residual) is taken while ||h||_inf is above tol_h; it
// corrects the rounding of the first.  The adjoint projects the upstream
// gradient onto null(A): grad = g - A^T S^{-1} A g.
//
// Layout: one workgroup of kBcWaves wavefronts per sample; wavefront w takes
// slabs w, w + kBcWaves, ...; lane l holds x = l, l + 64, ... of a slab in
// XR registers (the class: 64 XR >= nx, XR in {1, 2, 4, 8}), so the slab is
// read once from HBM and written once.  Every load is unconditional (lanes
// past the slab's end read its last value, masked where used) and up to
// four of the wavefront's next slabs are in flight while it works on the
// current one.  The kernel is HBM-bound on compulsory bytes.
#include "snap_device.hpp"

namespace snap {

namespace {

constexpr int kBcWaves = 16;
constexpr int kBcMaxX = 8;        // nx <= 512

struct BcRows {
  double dx, rdx, uL, m0, det;     // det = (nx - 1) dx^2 of the upper 2 x 2 block
  int nx;
};

// multipliers of one slab's rows from its residual (r_D, r_M, r_N)
__device__ __forceinline__ void bc_solve(const BcRows& R, double rD, double rM, double rN, double& lD,
                                         double& lM, double& lN) {
  const double s11 = R.nx * R.dx * R.dx;
  lD = (s11 * rD - R.dx * rM) / R.det;
  lM = (rM - R.dx * rD) / R.det;
  lN = 0.5 * rN * R.dx * R.dx;
}

// value at x of a slab held in registers, on every lane (x = lane + 64 j:
// read from lane x % 64 of register x / 64)
template <int XR>
__device__ __forceinline__ double bc_at(const double* v, int x) {
  double r = v[0];
#pragma unroll
  for (int j = 1; j < XR; ++j)
    if (x >= kWave * j) r = v[j];          // x is uniform: a scalar branch
  const int l = x & (kWave - 1);
  const int lo = __builtin_amdgcn_readlane(__double2loint(r), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(r), l);
  return __hiloint2double(hi, lo);
}

// residual of one slab held in registers (v[j] = u at x = lane + 64 j; zero
// past the slab's end): one wavefront sum for the mass, lane reads for the
// boundary values
template <int XR>
__device__ __forceinline__ void bc_residual(const BcRows& R, const double* v, int lane, bool homog,
                                            double& rD, double& rM, double& rN) {
  double s = 0.0;
#pragma unroll
  for (int j = 0; j < XR; ++j) s += v[j];
  s = wave_sum(s);
  const double a = bc_at<XR>(v, 0), bm = bc_at<XR>(v, R.nx - 2), bl = bc_at<XR>(v, R.nx - 1);
  rD = homog ? a : a - R.uL;
  rM = homog ? R.dx * s : R.dx * s - R.m0;
  rN = (bl - bm) * R.rdx;
}

// v -= A^T lam on the slab in registers (entries past the slab's end stay 0)
template <int XR>
__device__ __forceinline__ void bc_apply(const BcRows& R, double* v, int lane, double lD, double lM, double lN) {
#pragma unroll
  for (int j = 0; j < XR; ++j) {
    const int x = lane + kWave * j;
    double d = R.dx * lM;
    if (x == 0) d += lD;
    if (x == R.nx - 2) d -= lN * R.rdx;
    if (x == R.nx - 1) d += lN * R.rdx;
    if (x < R.nx) v[j] -= d;
  }
}

template <int XR>
__global__ __launch_bounds__(kBcWaves * kWave) void bc_kernel(KernelArgs A) {
  const int sid = A.order[blockIdx.x];
  const snap_sample_desc D = A.descs[sid];
  const int lane = threadIdx.x & (kWave - 1);
  const int w = threadIdx.x / kWave;
  __shared__ double red[kBcWaves][3];
  __shared__ int itmax[kBcWaves];

  BcRows R;
  R.nx = D.nx;
  R.dx = D.dx;
  R.rdx = 1.0 / D.dx;
  R.det = (D.nx - 1) * D.dx * D.dx;
  R.uL = A.backward ? 0.0 : A.aux[D.aux_off];
  R.m0 = A.backward ? 0.0 : A.aux[D.aux_off + 1];
  const int nt = D.nt, nx = D.nx;
  const int64_t vo = D.var_off, ro = D.row_off;
  const double* src = A.backward ? A.grad_u : A.uhat;
  double* dst = A.backward ? A.grad_uhat : A.u;
  const int max_it = A.opt.max_newton;

  double hmax = 0.0, smax = 0.0, umax = 0.0;
  int iters = 0, nonfin = 0;
  // unconditional loads: a slab past the last reads the last, a lane past the
  // slab's end its last value (never stored; masked in the sums).  Wavefront
  // w's slabs are k = w + kBcWaves i; kDepth of them are in flight at once
  // (whole rounds with one loop exit, so each wait covers one slab's loads).
  constexpr int kDepth = XR <= 2 ? 4 : (XR == 4 ? 2 : 1);
  auto load = [&](int i, double* dst) {
    const double* in = src + vo + (int64_t)min(w + kBcWaves * i, nt - 1) * nx;
#pragma unroll
    for (int j = 0; j < XR; ++j) dst[j] = in[min(lane + kWave * j, nx - 1)];
  };
  const int cnt = w < nt ? (nt - 1 - w) / kBcWaves + 1 : 0;   // this wavefront's slabs
  double stg[kDepth][XR];
#pragma unroll
  for (int b = 0; b < kDepth; ++b) load(b, stg[b]);
  for (int i0 = 0; i0 < cnt; i0 += kDepth) {
#pragma unroll
    for (int b = 0; b < kDepth; ++b) {
      const int i = i0 + b;
      if (i < cnt) {
        const int k = w + kBcWaves * i;
        double v[XR], v0[XR];
#pragma unroll
        for (int j = 0; j < XR; ++j) {
          const int x = lane + kWave * j;
          v[j] = x < nx ? stg[b][j] : 0.0;
          v0[j] = v[j];
          umax = fmax(umax, fabs(v[j]));
          nonfin |= !finite(v[j]);
        }
        double LD = 0.0, LM = 0.0, LN = 0.0, rD, rM, rN;
        bc_residual<XR>(R, v, lane, A.backward != 0, rD, rM, rN);
        int it = 0;
        // Newton steps on the slab (the first solves it; later ones correct rounding)
        while (it < max_it && (it == 0 || fmax(fabs(rD), fmax(fabs(rM), fabs(rN))) > A.opt.tol_h)) {
          double lD, lM, lN;
          bc_solve(R, rD, rM, rN, lD, lM, lN);
          bc_apply<XR>(R, v, lane, lD, lM, lN);
          LD += lD; LM += lM; LN += lN;
          bc_residual<XR>(R, v, lane, A.backward != 0, rD, rM, rN);
          ++it;
        }
        iters = max(iters, it);
        double* out = dst + vo + (int64_t)k * nx;
        double st = 0.0;
#pragma unroll
        for (int j = 0; j < XR; ++j) {
          const int x = lane + kWave * j;
          if (x < nx) {
            out[x] = v[j];
            // stationarity u - u_hat + A^T lam (forward)
            double at = R.dx * LM;
            if (x == 0) at += LD;
            if (x == nx - 2) at -= LN * R.rdx;
            if (x == nx - 1) at += LN * R.rdx;
            st = fmax(st, fabs(v[j] - v0[j] + at));
          }
        }
        if (!A.backward && lane == 0) {
          A.lam[ro + k] = LD;
          A.lam[ro + nt + k] = LM;
          A.lam[ro + 2 * nt + k] = LN;
        }
        hmax = fmax(hmax, fmax(fabs(rD), fmax(fabs(rM), fabs(rN))));
        smax = fmax(smax, wave_max(st));
      }
      load(i + kDepth, stg[b]);
    }
  }
  // per-sample stats (forward: status from the final residuals)
  umax = wave_max(umax);
  const double nf = wave_max((double)nonfin);
  if (lane == 0) {
    red[w][0] = hmax;
    red[w][1] = smax;
    red[w][2] = fmax(umax, nf > 0.0 ? __builtin_inf() : 0.0);
    itmax[w] = iters;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double h = 0.0, s = 0.0, um = 0.0;
    int it = 0;
    for (int q = 0; q < kBcWaves; ++q) {
      h = fmax(h, red[q][0]);
      s = fmax(s, red[q][1]);
      um = fmax(um, red[q][2]);
      it = max(it, itmax[q]);
    }
    snap_sample_stats out{};
    out.newton_iters = it;
    out.h_inf = h;
    out.stat_inf = s;
    if (!finite(um) || !finite(h) || !finite(s))
      out.status = SNAP_ST_NONFINITE;
    else if (A.backward || (h <= A.opt.tol_h && s <= A.opt.tol_s * (1.0 + um)))
      out.status = SNAP_ST_CONVERGED;
    else
      out.status = SNAP_ST_MAX_ITER;
    A.stats[sid] = out;
  }
}

}  // namespace

bool bc_supported(int nx, int ny, int nt) { return ny == 1 && nx >= 3 && nx <= kWave * kBcMaxX && nt >= 1; }

// x registers per lane for a slab of nx points
int bc_class(int nx) { return nx <= kWave ? 1 : nx <= 2 * kWave ? 2 : nx <= 4 * kWave ? 4 : 8; }

int bc_launch(const KernelArgs& a, int cls, hipStream_t st) {
  if (a.count <= 0) return 0;
  const dim3 grid(a.count), block(kBcWaves * kWave);
  switch (cls) {
    case 1: hipLaunchKernelGGL(bc_kernel<1>, grid, block, 0, st, a); break;
    case 2: hipLaunchKernelGGL(bc_kernel<2>, grid, block, 0, st, a); break;
    case 4: hipLaunchKernelGGL(bc_kernel<4>, grid, block, 0, st, a); break;
    case 8: hipLaunchKernelGGL(bc_kernel<8>, grid, block, 0, st, a); break;
    default: return SNAP_EUNSUPPORTED;
  }
  return hipGetLastError() == hipSuccess ? 0 : SNAP_EHIP;
}

}  // namespace snap
