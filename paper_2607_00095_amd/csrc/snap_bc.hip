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
// Layout: one workgroup of kBcWaves wavefronts per sample.  A group of G
// lanes owns a slab (G = 16, a DPP row, for nx <= 128; G = 64, the whole
// wavefront, above), lane p of the group holds x = p, p + G, ... in XR
// registers (G XR >= nx), so a slab is read once from HBM and written once
// and a wavefront projects 64 / G slabs at a time.  Group sums are DPP row
// rotations (G = 16) or the wavefront reduction (G = 64); the boundary values
// are group sums of masked values.  Every load is unconditional (lanes past
// the slab's end, and groups past the last slab, read valid addresses and are
// masked where used) and the next kDepth rounds of slabs are in flight while
// the wavefront works on the current one.  The kernel is HBM-bound on
// compulsory bytes.
#include "snap_device.hpp"

namespace snap {

namespace {

constexpr int kBcWaves = 8;

struct BcRows {
  double dx, rdx, uL, m0, det;     // det = (nx - 1) dx^2 of the upper 2 x 2 block
  int nx;
};

// sum over the G lanes of a group, the same in every lane of the group
template <int G>
__device__ __forceinline__ double group_sum(double x) {
  if constexpr (G == 16) {
    x += dpp_d<0x128, 0xf, true>(x);   // row_ror:8
    x += dpp_d<0x124, 0xf, true>(x);   // row_ror:4
    x += dpp_d<0x122, 0xf, true>(x);   // row_ror:2
    x += dpp_d<0x121, 0xf, true>(x);   // row_ror:1
    return x;
  } else {
    return wave_sum(x);
  }
}

// multipliers of one slab's rows from its residual (r_D, r_M, r_N)
__device__ __forceinline__ void bc_solve(const BcRows& R, double rD, double rM, double rN, double& lD,
                                         double& lM, double& lN) {
  const double s11 = R.nx * R.dx * R.dx;
  lD = (s11 * rD - R.dx * rM) / R.det;
  lM = (rM - R.dx * rD) / R.det;
  lN = 0.5 * rN * R.dx * R.dx;
}

// residual of the group's slab held in registers (v[j] = u at x = p + G j;
// zero past the slab's end)
template <int G, int XR>
__device__ __forceinline__ void bc_residual(const BcRows& R, const double* v, int p, bool homog,
                                            double& rD, double& rM, double& rN) {
  double s = 0.0, a = 0.0, bm = 0.0, bl = 0.0;
#pragma unroll
  for (int j = 0; j < XR; ++j) {
    const int x = p + G * j;
    s += v[j];
    a += x == 0 ? v[j] : 0.0;
    bm += x == R.nx - 2 ? v[j] : 0.0;
    bl += x == R.nx - 1 ? v[j] : 0.0;
  }
  s = group_sum<G>(s);
  a = group_sum<G>(a);
  bm = group_sum<G>(bm);
  bl = group_sum<G>(bl);
  rD = homog ? a : a - R.uL;
  rM = homog ? R.dx * s : R.dx * s - R.m0;
  rN = (bl - bm) * R.rdx;
}

// A^T lam at x
__device__ __forceinline__ double bc_at(const BcRows& R, int x, double lD, double lM, double lN) {
  double d = R.dx * lM;
  if (x == 0) d += lD;
  if (x == R.nx - 2) d -= lN * R.rdx;
  if (x == R.nx - 1) d += lN * R.rdx;
  return d;
}

template <int G, int XR>
__global__ __launch_bounds__(kBcWaves * kWave) void bc_kernel(KernelArgs A) {
  constexpr int SPW = kWave / G;                         // slabs a wavefront projects at once
  constexpr int kDepth = XR <= 2 ? 4 : (XR == 4 ? 2 : 1);
  const int sid = A.order[blockIdx.x];
  const snap_sample_desc D = A.descs[sid];
  const int lane = threadIdx.x & (kWave - 1);
  const int w = threadIdx.x / kWave;
  const int p = lane % G, grp = lane / G;
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

  // round i of wavefront w: slabs SPW (w + kBcWaves i) + grp; unconditional
  // loads (past the last slab: the last slab; past the slab's end: its last
  // value), masked where used
  const int rounds = (nt + SPW - 1) / SPW;
  const int cnt = w < rounds ? (rounds - 1 - w) / kBcWaves + 1 : 0;
  auto slab_of = [&](int i) { return SPW * (w + kBcWaves * i) + grp; };
  auto load = [&](int i, double* dstv) {
    const double* in = src + vo + (int64_t)min(slab_of(i), nt - 1) * nx;
#pragma unroll
    for (int j = 0; j < XR; ++j) dstv[j] = in[min(p + G * j, nx - 1)];
  };
  double hmax = 0.0, smax = 0.0, umax = 0.0;
  int iters = 0, nonfin = 0;
  double stg[kDepth][XR];
#pragma unroll
  for (int b = 0; b < kDepth; ++b) load(b, stg[b]);
  // whole rounds of kDepth stages with one loop exit, so each wait covers one
  // stage's loads
  for (int i0 = 0; i0 < cnt; i0 += kDepth) {
#pragma unroll
    for (int b = 0; b < kDepth; ++b) {
      const int i = i0 + b;
      if (i < cnt) {
        const int k = slab_of(i);
        const bool live = k < nt;
        double v[XR], v0[XR];
#pragma unroll
        for (int j = 0; j < XR; ++j) {
          v[j] = (live && p + G * j < nx) ? stg[b][j] : 0.0;
          v0[j] = v[j];
          umax = fmax(umax, fabs(v[j]));
          nonfin |= !finite(v[j]);
        }
        double LD = 0.0, LM = 0.0, LN = 0.0, rD, rM, rN;
        bc_residual<G, XR>(R, v, p, A.backward != 0, rD, rM, rN);
        double rmax = live ? fmax(fabs(rD), fmax(fabs(rM), fabs(rN))) : 0.0;
        int it = 0;
        // Newton steps on the slabs (the first solves them; later ones correct
        // rounding), while any group of the wavefront is above the tolerance
        while (it < max_it && (it == 0 || wave_max(rmax) > A.opt.tol_h)) {
          double lD, lM, lN;
          bc_solve(R, rD, rM, rN, lD, lM, lN);
#pragma unroll
          for (int j = 0; j < XR; ++j) {
            const int x = p + G * j;
            if (x < nx) v[j] -= bc_at(R, x, lD, lM, lN);
          }
          LD += lD; LM += lM; LN += lN;
          bc_residual<G, XR>(R, v, p, A.backward != 0, rD, rM, rN);
          rmax = live ? fmax(fabs(rD), fmax(fabs(rM), fabs(rN))) : 0.0;
          ++it;
        }
        iters = max(iters, it);
        if (live) {
          double* out = dst + vo + (int64_t)k * nx;
#pragma unroll
          for (int j = 0; j < XR; ++j) {
            const int x = p + G * j;
            if (x < nx) {
              out[x] = v[j];
              // stationarity u - u_hat + A^T lam
              smax = fmax(smax, fabs(v[j] - v0[j] + bc_at(R, x, LD, LM, LN)));
            }
          }
          if (!A.backward && p == 0) {
            A.lam[ro + k] = LD;
            A.lam[ro + nt + k] = LM;
            A.lam[ro + 2 * nt + k] = LN;
          }
          hmax = fmax(hmax, rmax);
        }
      }
      load(i + kDepth, stg[b]);
    }
  }
  // per-sample stats (forward: status from the final residuals)
  hmax = wave_max(hmax);
  smax = wave_max(smax);
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

bool bc_supported(int nx, int ny, int nt) { return ny == 1 && nx >= 3 && nx <= 512 && nt >= 1; }

// launch class: lanes per slab and x registers per lane (G = 16 up to
// nx = 128: 1, 2, 4, 8; G = 64 above: 104 (nx <= 256), 108)
int bc_class(int nx) {
  if (nx <= 128) return nx <= 16 ? 1 : nx <= 32 ? 2 : nx <= 64 ? 4 : 8;
  return nx <= 256 ? 104 : 108;
}

int bc_launch(const KernelArgs& a, int cls, hipStream_t st) {
  if (a.count <= 0) return 0;
  const dim3 grid(a.count), block(kBcWaves * kWave);
  switch (cls) {
    case 1: hipLaunchKernelGGL((bc_kernel<16, 1>), grid, block, 0, st, a); break;
    case 2: hipLaunchKernelGGL((bc_kernel<16, 2>), grid, block, 0, st, a); break;
    case 4: hipLaunchKernelGGL((bc_kernel<16, 4>), grid, block, 0, st, a); break;
    case 8: hipLaunchKernelGGL((bc_kernel<16, 8>), grid, block, 0, st, a); break;
    case 104: hipLaunchKernelGGL((bc_kernel<64, 4>), grid, block, 0, st, a); break;
    case 108: hipLaunchKernelGGL((bc_kernel<64, 8>), grid, block, 0, st, a); break;
    default: return SNAP_EUNSUPPORTED;
  }
  return hipGetLastError() == hipSuccess ? 0 : SNAP_EHIP;
}

}  // namespace snap
