// Slab-row families (mass + IC, Fisher-KPP) on wide grids (128 < Nx <= 256),
// where one lane cannot keep both the field and the Newton step of its share of
// the sample in registers: every slab sum is a reduction over a whole
// wavefront.  Wavefront w owns time slabs w, w+8, ...; lane l owns
// x = l, l+64, ....  The mathematics (Schur form of the Newton-KKT system of
// Appendix B, IC elimination, tridiagonal solve by parallel cyclic reduction,
// l1-merit line search) is the one of the grouped kernel for Nx <= 128 in
// snap_slab.hip, which documents it.
#include "snap_device.hpp"

namespace snap {
namespace {

constexpr int kSlabWaves = 8;
constexpr int kSlabThreads = kSlabWaves * kWave;
constexpr int kMaxNt = 128;

template <typename TS>
struct PcrBuf {
  TS a[2][kMaxNt], b[2][kMaxNt], c[2][kMaxNt], d[2][kMaxNt];
};

// Parallel cyclic reduction of the symmetric tridiagonal system
// diag Td[0..n), off-diagonal To[k] = T_{k,k+1}, right-hand side rhs, by ONE
// wavefront (n <= 128, two equations per lane), in precision TS.  The result is
// written to x (double, LDS).
template <typename TS>
__device__ void pcr_solve(int n, const double* Td, const double* To, const double* rhs,
                          double* x, PcrBuf<TS>& B) {
  const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    int j = lane + kWave * e;
    if (j < n) {
      B.a[0][j] = j > 0 ? (TS)To[j - 1] : (TS)0;
      B.b[0][j] = (TS)Td[j];
      B.c[0][j] = j < n - 1 ? (TS)To[j] : (TS)0;
      B.d[0][j] = (TS)rhs[j];
    }
  }
  wave_sync();
  int cur = 0;
  for (int s = 1; s < n; s <<= 1) {
    TS na[2], nb[2], nc[2], nd[2];
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      int j = lane + kWave * e;
      if (j < n) {
        TS aj = B.a[cur][j], bj = B.b[cur][j], cj = B.c[cur][j], dj = B.d[cur][j];
        TS an = 0, cn = 0;
        if (j - s >= 0) {
          TS al = -aj / B.b[cur][j - s];
          an = al * B.a[cur][j - s];
          bj += al * B.c[cur][j - s];
          dj += al * B.d[cur][j - s];
        }
        if (j + s < n) {
          TS ga = -cj / B.b[cur][j + s];
          cn = ga * B.c[cur][j + s];
          bj += ga * B.a[cur][j + s];
          dj += ga * B.d[cur][j + s];
        }
        na[e] = an; nb[e] = bj; nc[e] = cn; nd[e] = dj;
      }
    }
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      int j = lane + kWave * e;
      if (j < n) {
        B.a[cur ^ 1][j] = na[e]; B.b[cur ^ 1][j] = nb[e];
        B.c[cur ^ 1][j] = nc[e]; B.d[cur ^ 1][j] = nd[e];
      }
    }
    wave_sync();
    cur ^= 1;
  }
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    int j = lane + kWave * e;
    if (j < n) x[j] = (double)(B.d[cur][j] / B.b[cur][j]);
  }
  wave_sync();
}

struct SlabShared {
  // per-slab sums: S1 = sum u, S2 = sum u(1-u), Sd = sum g, Sa2 = sum a^2, Sa = sum a,
  // Sad = sum a*g with g the stationarity residual
  double S1[kMaxNt], S2[kMaxNt], Sd[kMaxNt], Sa2[kMaxNt], Sa[kMaxNt], Sad[kMaxNt];
  double W[kMaxNt];      // W_k per slab
  double lam[kMaxNt];    // current multipliers of the slab rows
  double lamp[kMaxNt];   // Newton multipliers lam+
  double Td[kMaxNt], To[kMaxNt], r[kMaxNt], res[kMaxNt], dx[kMaxNt];
  double red[kSlabWaves][4];
  double scal[16];
  int flag[4];
};

// Row-k coefficient on slab k (derivative of row k w.r.t. u(x,k)).
__device__ __forceinline__ double coef_a(bool f2, double c, double uu) {
  return f2 ? (-1.0 - c * (1.0 - 2.0 * uu)) : 0.0;
}

template <int SPW, int XPL, bool UREG, typename TS>
__global__ __launch_bounds__(kSlabThreads, 1) void slab_wide_kernel(KernelArgs A) {
  const int sid = A.order[blockIdx.x];
  const snap_sample_desc D = A.descs[sid];
  const int nx = D.nx, nt = D.nt, nr = nt - 1;
  const bool f2 = (D.family == SNAP_FISHER_KPP);
  const double c = f2 ? D.dt * D.p0 : 0.0;
  const double wfloor = 0.1;
  const int lane = threadIdx.x & (kWave - 1);
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);   // wave-uniform
  const bool bwd = A.backward != 0;

  __shared__ SlabShared sh;
  __shared__ PcrBuf<TS> pcr;

  const double* uhat_g = A.uhat + D.var_off;
  const double* aux = A.aux + D.aux_off;
  const double m0 = f2 ? 0.0 : aux[nx];

  double u[SPW][XPL];
  double uh[UREG ? SPW : 1][UREG ? XPL : 1];
  double gic[XPL], lamic[XPL], lampic[XPL];

  auto slab_of = [&](int s) { return w + kSlabWaves * s; };
  auto xof = [&](int j) { return lane + kWave * j; };
  // u_hat as seen by the step: forward -> input u_hat; backward -> u* + grad_u,
  // so that u - u_hat_eff = -grad_u and the step formula yields the adjoint.
  auto uhat_at = [&](int s, int j) -> double {
    if constexpr (UREG) {
      return uh[s][j];
    } else {
      int64_t idx = (int64_t)slab_of(s) * nx + xof(j);
      return bwd ? (A.u[D.var_off + idx] + A.grad_u[D.var_off + idx]) : uhat_g[idx];
    }
  };

  // ---------------------------------------------------------------- load
  double umax = 0.0;
  bool nonfinite = false;
#pragma unroll
  for (int s = 0; s < SPW; ++s) {
    const int k = slab_of(s);
#pragma unroll
    for (int j = 0; j < XPL; ++j) {
      const int x = xof(j);
      double uu = 0.0, hh = 0.0;
      if (k < nt && x < nx) {
        int64_t idx = (int64_t)k * nx + x;
        if (bwd) {
          uu = A.u[D.var_off + idx];
          hh = uu + A.grad_u[D.var_off + idx];
        } else {
          hh = uhat_g[idx];
          uu = hh;
        }
        umax = fmax(umax, fabs(hh));
        nonfinite |= !finite(hh) || !finite(uu);
      }
      u[s][j] = uu;
      if constexpr (UREG) uh[s][j] = hh;
    }
  }
#pragma unroll
  for (int j = 0; j < XPL; ++j) {
    const int x = xof(j);
    gic[j] = (w == 0 && x < nx) ? aux[x] : 0.0;
    lamic[j] = (bwd && w == 0 && x < nx) ? A.lam[D.row_off + x] : 0.0;
    lampic[j] = 0.0;
  }
  int floored = 0;   // adjoint: exact W below the floor somewhere
  for (int k = threadIdx.x; k < kMaxNt; k += kSlabThreads) {
    double l = (bwd && k < nr) ? A.lam[D.row_off + nx + k] : 0.0;
    sh.lam[k] = l;
    sh.lamp[k] = 0.0;
    double wk = (k < nr) ? 1.0 + 2.0 * c * l : 1.0;
    floored |= k < nr && wk < wfloor;
    sh.W[k] = fmax(wk, wfloor);
  }
  floored = __syncthreads_or(floored);
  if (bwd) {
    // W is taken at lam*; the adjoint right-hand side uses J W^{-1} grad_u only,
    // so the multipliers entering the stationarity residual are zero
    lds_barrier();
    for (int k = threadIdx.x; k < kMaxNt; k += kSlabThreads) sh.lam[k] = 0.0;
#pragma unroll
    for (int j = 0; j < XPL; ++j) lamic[j] = 0.0;
  }
  {
    double mx = wave_max(umax);
    int nf = __any(nonfinite) ? 1 : 0;
    if (lane == 0) { sh.red[w][0] = mx; sh.red[w][1] = (double)nf; }
  }
  lds_barrier();
  double uscale = 0.0, nfin = 0.0;
  for (int q = 0; q < kSlabWaves; ++q) { uscale = fmax(uscale, sh.red[q][0]); nfin += sh.red[q][1]; }
  uscale += 1.0;
  lds_barrier();

  double mu = 0.0;
  int iters = 0, backtracks = 0, refines = 0, status = SNAP_ST_MAX_ITER;
  double hinf = 0.0, stinf = 0.0;
  if (nfin > 0.0) status = SNAP_ST_NONFINITE;
  const int max_it = bwd ? 1 : A.opt.max_newton;

  for (int it = 0; status != SNAP_ST_NONFINITE; ++it) {
    // ------------------------------------------------ pass 1: slab sums
    double st_w = 0.0;
#pragma unroll
    for (int s = 0; s < SPW; ++s) {
      const int k = slab_of(s);
      if (k >= nt) continue;                       // uniform over the wavefront
      const double lk = (k < nr) ? sh.lam[k] : 0.0;
      const double lkm = (k >= 1) ? sh.lam[k - 1] : 0.0;
      // a_k(x) = d row_k / d u(x,k) = a0 + 2c u(x,k) is affine in u, so four
      // sums per slab give every slab quantity: sum u, sum u^2, sum g, sum u g
      double Su = 0, Suu = 0, Sg = 0, Sug = 0;
#pragma unroll
      for (int j = 0; j < XPL; ++j) {
        const int x = xof(j);
        if (x < nx) {
          const double uu = u[s][j];
          const double d = uu - uhat_at(s, j);
          const double a = (k < nr) ? coef_a(f2, c, uu) : 0.0;
          // stationarity residual g = u - u_hat + J^T lam; the Newton system is
          // solved for the multiplier increment with right-hand side
          // h - J W^{-1} g, which vanishes at the solution
          const double gg = d + a * lk + (k >= 1 ? lkm : 0.0) + (k == 0 ? lamic[j] : 0.0);
          Su += uu; Suu += uu * uu; Sg += gg; Sug += uu * gg;
          st_w = fmax(st_w, fabs(gg));
        }
      }
      Su = wave_sum(Su); Suu = wave_sum(Suu); Sg = wave_sum(Sg); Sug = wave_sum(Sug);
      if (lane == 0) {
        const double a0 = (k < nr && f2) ? -1.0 - c : 0.0, a1 = (k < nr && f2) ? 2.0 * c : 0.0;
        const double cnt = (double)nx;
        sh.S1[k] = Su; sh.S2[k] = Su - Suu; sh.Sd[k] = Sg;
        sh.Sa[k] = a0 * cnt + a1 * Su;
        sh.Sa2[k] = a0 * a0 * cnt + 2.0 * a0 * a1 * Su + a1 * a1 * Suu;
        sh.Sad[k] = a0 * Sg + a1 * Sug;
      }
      // one slab's reductions at a time (bounds register pressure)
      __builtin_amdgcn_sched_barrier(0);
    }
    // IC rows live on slab 0, owned by wavefront 0 (s = 0)
    double ric[XPL];
    if (w == 0) {
      double sar = 0.0, hicmax = 0.0, hic1 = 0.0;
      const double W0 = sh.W[0];
#pragma unroll
      for (int j = 0; j < XPL; ++j) {
        const int x = xof(j);
        ric[j] = 0.0;
        if (x < nx) {
          const double uu = u[0][j];
          const double a0 = (nr > 0) ? coef_a(f2, c, uu) : 0.0;
          const double gg = uu - uhat_at(0, j) + lamic[j] + (nr > 0 ? a0 * sh.lam[0] : 0.0);
          const double hic = bwd ? 0.0 : uu - gic[j];
          ric[j] = hic - gg / W0;
          sar += a0 * ric[j];
          hicmax = fmax(hicmax, fabs(hic));
          hic1 += fabs(hic);
        }
      }
      sar = wave_sum(sar); hicmax = wave_max(hicmax); hic1 = wave_sum(hic1);
      if (lane == 0) { sh.scal[0] = sar; sh.scal[1] = hicmax; sh.scal[2] = hic1; }
    }
    st_w = wave_max(st_w);
    if (lane == 0) sh.red[w][0] = st_w;
    lds_barrier();

    // ------------------------------------------------ wavefront 0: rows, test, solve
    if (w == 0) {
      double hmax = sh.scal[1], h1 = sh.scal[2];
      for (int k = lane; k < nr; k += kWave) {
        double hk = bwd ? 0.0
                        : (f2 ? sh.S1[k + 1] - sh.S1[k] - c * sh.S2[k] : sh.S1[k + 1] - m0);
        const double Wk = sh.W[k], Wk1 = sh.W[k + 1];
        double rk = hk - (sh.Sad[k] / Wk + sh.Sd[k + 1] / Wk1);
        if (k == 0) rk -= sh.scal[0];
        sh.r[k] = rk;
        sh.Td[k] = (k == 0 ? 0.0 : sh.Sa2[k] / Wk) + (double)nx / Wk1;
        sh.To[k] = (k + 1 < nr) ? sh.Sa[k + 1] / Wk1 : 0.0;
        hmax = fmax(hmax, fabs(hk));
        h1 += fabs(hk);
        if (!finite(hk)) hmax = __builtin_nan("");
      }
      hmax = wave_max(hmax);
      h1 = wave_sum(h1);
      double stmax = 0.0;
      for (int q = 0; q < kSlabWaves; ++q) stmax = fmax(stmax, sh.red[q][0]);
      int done = 0;
      if (!bwd) {
        hinf = hmax; stinf = stmax;
        if (!finite(hmax) || !finite(stmax)) done = 2;
        else if (hmax <= A.opt.tol_h && stmax <= A.opt.tol_s * uscale) done = 1;
        else if (it >= max_it) done = 3;
      }
      if (lane == 0) { sh.flag[0] = done; sh.scal[3] = h1; }
      if (!done && nr > 0) {
        if constexpr (sizeof(TS) == sizeof(double)) {
          pcr_solve<TS>(nr, sh.Td, sh.To, sh.r, sh.lamp, pcr);
        } else {
          // float32 solve + float64 residual refinement
          pcr_solve<TS>(nr, sh.Td, sh.To, sh.r, sh.lamp, pcr);
          double rn = 0.0;
          for (int k = lane; k < nr; k += kWave) rn = fmax(rn, fabs(sh.r[k]));
          rn = wave_max(rn);
          for (int ref = 0; ref < 4; ++ref) {
            double resmax = 0.0;
            for (int k = lane; k < nr; k += kWave) {
              double tx = sh.Td[k] * sh.lamp[k];
              if (k > 0) tx += sh.To[k - 1] * sh.lamp[k - 1];
              if (k + 1 < nr) tx += sh.To[k] * sh.lamp[k + 1];
              sh.res[k] = sh.r[k] - tx;
              resmax = fmax(resmax, fabs(sh.res[k]));
            }
            resmax = wave_max(resmax);
            wave_sync();
            const double target = bwd ? 1e-15 * rn
                                      : (hinf > 1e-6 ? 1e-6 * rn : fmax(1e-15 * rn, 0.1 * A.opt.tol_h));
            if (!(resmax > target)) break;
            pcr_solve<TS>(nr, sh.Td, sh.To, sh.res, sh.dx, pcr);
            for (int k = lane; k < nr; k += kWave) sh.lamp[k] += sh.dx[k];
            wave_sync();
            ++refines;
          }
        }
      }
      if (!done) {
        // sh.lamp holds the increment; form lam+ = lam + dlam
        const double l0 = nr > 0 ? sh.lamp[0] : 0.0;
        const double W0 = sh.W[0];
#pragma unroll
        for (int j = 0; j < XPL; ++j) {
          const double a0 = (nr > 0) ? coef_a(f2, c, u[0][j]) : 0.0;
          lampic[j] = lamic[j] + (W0 * ric[j] - a0 * l0);
        }
        wave_sync();
        for (int k = lane; k < nr; k += kWave) sh.lamp[k] += sh.lam[k];
      }
    }
    lds_barrier();
    const int done = sh.flag[0];
    if (done) {
      status = done == 1 ? SNAP_ST_CONVERGED : (done == 2 ? SNAP_ST_NONFINITE : SNAP_ST_MAX_ITER);
      break;
    }

    // ------------------------------------------------ step p = -(d + J^T lam+)/W
    // backward: the step is the adjoint; write it and stop
    auto step_at = [&](int s, int j, int k, double uu) -> double {
      const double d = uu - uhat_at(s, j);
      const double a = (k < nr) ? coef_a(f2, c, uu) : 0.0;
      double jt = d + a * ((k < nr) ? sh.lamp[k] : 0.0) + (k >= 1 ? sh.lamp[k - 1] : 0.0)
                + (k == 0 ? lampic[j] : 0.0);
      return -jt / sh.W[k];
    };
    if (bwd) {
#pragma unroll
      for (int s = 0; s < SPW; ++s) {
        const int k = slab_of(s);
        if (k >= nt) continue;
#pragma unroll
        for (int j = 0; j < XPL; ++j) {
          const int x = xof(j);
          if (x < nx) A.grad_uhat[D.var_off + (int64_t)k * nx + x] = step_at(s, j, k, u[s][j]);
        }
      }
      status = floored ? SNAP_ST_HESSIAN_FLOOR : SNAP_ST_CONVERGED;
      break;
    }

    // the step, once, into registers (the line search and the update reuse it)
    double pst[SPW][XPL];
#pragma unroll
    for (int s = 0; s < SPW; ++s) {
      const int k = slab_of(s);
#pragma unroll
      for (int j = 0; j < XPL; ++j)
        pst[s][j] = (k < nt && xof(j) < nx) ? step_at(s, j, k, u[s][j]) : 0.0;
    }

    // merit phi = 1/2||u - u_hat||^2 + mu*||h||_1 and its directional derivative
    double lmax = 0.0;
    if (w == 0) {
      double lm = 0.0;
#pragma unroll
      for (int j = 0; j < XPL; ++j) lm = fmax(lm, fabs(lampic[j]));
      for (int k = lane; k < nr; k += kWave) lm = fmax(lm, fabs(sh.lamp[k]));
      lm = wave_max(lm);
      if (lane == 0) sh.scal[4] = lm;
    }
    {
      double pp = 0.0, dd = 0.0;
#pragma unroll
      for (int s = 0; s < SPW; ++s) {
        const int k = slab_of(s);
        if (k >= nt) continue;
#pragma unroll
        for (int j = 0; j < XPL; ++j) {
          if (xof(j) < nx) {
            const double d = u[s][j] - uhat_at(s, j);
            const double p = pst[s][j];
            pp += p * p;
            dd += d * p;
          }
        }
      }
      pp = wave_sum(pp); dd = wave_sum(dd);
      if (lane == 0) { sh.red[w][1] = pp; sh.red[w][2] = dd; }
    }
    lds_barrier();
    lmax = fmax(lmax, sh.scal[4]);
    mu = fmax(mu, 1.1 * lmax + 1e-8);
    // the merit change along p is formed from differences (alpha d.p +
    // alpha^2/2 p.p + mu(||h_t||_1 - ||h||_1)), so rounding of the large sums
    // in phi itself never decides acceptance
    double pp = 0.0, dd = 0.0;
    for (int q = 0; q < kSlabWaves; ++q) { pp += sh.red[q][1]; dd += sh.red[q][2]; }
    const double h1_0 = sh.scal[3];
    const double dphi = dd - mu * h1_0;
    lds_barrier();

    // ------------------------------------------------ backtracking line search
    double alpha = 1.0;
    int accepted = 0;
    for (int ls = 0; ls <= A.opt.max_ls; ++ls) {
#pragma unroll
      for (int s = 0; s < SPW; ++s) {
        const int k = slab_of(s);
        if (k >= nt) continue;
        double S1 = 0, S2 = 0;
#pragma unroll
        for (int j = 0; j < XPL; ++j) {
          if (xof(j) < nx) {
            const double ut = u[s][j] + alpha * pst[s][j];
            S1 += ut; S2 += ut * (1.0 - ut);
          }
        }
        S1 = wave_sum(S1); S2 = wave_sum(S2);
        if (lane == 0) { sh.S1[k] = S1; sh.S2[k] = S2; }
        __builtin_amdgcn_sched_barrier(0);
      }
      if (w == 0) {
        double hic1 = 0.0;
#pragma unroll
        for (int j = 0; j < XPL; ++j) {
          if (xof(j) < nx) {
            const double ut = u[0][j] + alpha * pst[0][j];
            hic1 += fabs(ut - gic[j]);
          }
        }
        hic1 = wave_sum(hic1);
        if (lane == 0) sh.scal[5] = hic1;
      }
      lds_barrier();
      if (w == 0) {
        double h1 = sh.scal[5];
        for (int k = lane; k < nr; k += kWave) {
          double hk = f2 ? sh.S1[k + 1] - sh.S1[k] - c * sh.S2[k] : sh.S1[k + 1] - m0;
          h1 += fabs(hk);
        }
        h1 = wave_sum(h1);
        const double dphi_t = alpha * dd + 0.5 * alpha * alpha * pp + mu * (h1 - h1_0);
        // local phase (||h||_inf <= 1e-6): full Newton steps; there the change of
        // ||h||_1 along p sits below the rounding of the row sums
        // (with W >= 0.1 the step is a descent direction of the merit unless
        // it is zero; a zero step is taken, any other must pass the test)
        int ok = (dphi_t <= 1e-4 * alpha * dphi) || !(pp > 0.0) || hinf <= 1e-6 ? 1 : 0;
        if (lane == 0) sh.flag[1] = ok;
      }
      lds_barrier();
      if (sh.flag[1]) { accepted = 1; break; }
      alpha *= 0.5;
      ++backtracks;
    }
    if (!accepted) {
      status = SNAP_ST_LS_FAIL;
      break;
    }
    // ------------------------------------------------ accept: u += alpha p, lam += alpha (lam+ - lam)
#pragma unroll
    for (int s = 0; s < SPW; ++s) {
      const int k = slab_of(s);
      if (k >= nt) continue;
#pragma unroll
      for (int j = 0; j < XPL; ++j)
        if (xof(j) < nx) u[s][j] += alpha * pst[s][j];
    }
    // every thread computed its step with the old u above; now update lam, W
    lds_barrier();
    if (w == 0) {
#pragma unroll
      for (int j = 0; j < XPL; ++j) lamic[j] += alpha * (lampic[j] - lamic[j]);
    }
    for (int k = threadIdx.x; k < nr; k += kSlabThreads) {
      double l = sh.lam[k] + alpha * (sh.lamp[k] - sh.lam[k]);
      sh.lam[k] = l;
      sh.W[k] = fmax(1.0 + 2.0 * c * l, wfloor);
    }
    ++iters;
    lds_barrier();
  }

  // ---------------------------------------------------------------- outputs
  if (!bwd) {
#pragma unroll
    for (int s = 0; s < SPW; ++s) {
      const int k = slab_of(s);
      if (k >= nt) continue;
#pragma unroll
      for (int j = 0; j < XPL; ++j) {
        const int x = xof(j);
        if (x < nx) A.u[D.var_off + (int64_t)k * nx + x] = u[s][j];
      }
    }
    if (w == 0) {
#pragma unroll
      for (int j = 0; j < XPL; ++j)
        if (xof(j) < nx) A.lam[D.row_off + xof(j)] = lamic[j];
    }
    for (int k = threadIdx.x; k < nr; k += kSlabThreads) A.lam[D.row_off + nx + k] = sh.lam[k];
  }
  if (threadIdx.x == 0) {
    snap_sample_stats st;
    st.status = status;
    st.newton_iters = iters;
    st.ls_backtracks = backtracks;
    st.refine_steps = refines;
    st.h_inf = bwd ? 0.0 : hinf;
    st.stat_inf = bwd ? 0.0 : stinf;
    A.stats[sid] = st;
  }
}

// ------------------------------------------------------------------ dispatch
using SlabLaunch = void (*)(const KernelArgs&, hipStream_t);

template <int SPW, int XPL, typename TS>
static void launch_slab(const KernelArgs& a, hipStream_t st) {
  constexpr bool ureg = SPW * XPL <= 26;
  hipLaunchKernelGGL((slab_wide_kernel<SPW, XPL, ureg, TS>), dim3(a.count), dim3(kSlabThreads), 0, st, a);
}

template <typename TS>
static SlabLaunch pick_slab(int spw, int xpl) {
#define SNAP_SLAB_CASE(S, X) if (spw <= S && xpl == X) return &launch_slab<S, X, TS>;
#define SNAP_SLAB_ROW(X) SNAP_SLAB_CASE(1, X) SNAP_SLAB_CASE(2, X) SNAP_SLAB_CASE(4, X) \
                         SNAP_SLAB_CASE(8, X) SNAP_SLAB_CASE(13, X) SNAP_SLAB_CASE(16, X)
  SNAP_SLAB_ROW(3) SNAP_SLAB_ROW(4)
#undef SNAP_SLAB_ROW
#undef SNAP_SLAB_CASE
  return nullptr;
}

}  // namespace

// Kernel class of a wide (nx, nt) shape: index of the (SPW, XPL) instantiation, or -1.
int slab_wide_class(int nx, int nt) {
  if (nt < 1 || nt > kMaxNt || nx <= 2 * kWave || nx > 4 * kWave) return -1;
  const int spw = (nt + kSlabWaves - 1) / kSlabWaves;
  const int xpl = (nx + kWave - 1) / kWave;
  static const int spws[] = {1, 2, 4, 8, 13, 16};
  for (int i = 0; i < 6; ++i)
    if (spw <= spws[i]) return i * 2 + (xpl - 3);
  return -1;
}

// Host entry used by the plan: one workgroup per listed sample; every sample
// of the launch belongs to kernel class `cls` (shapes may differ).
int slab_wide_launch(const KernelArgs& a, int cls, bool mixed, hipStream_t st) {
  if (a.count == 0) return 0;
  static const int spws[] = {1, 2, 4, 8, 13, 16};
  if (cls < 0 || cls >= 12) return SNAP_EUNSUPPORTED;
  const int spw = spws[cls / 2], xpl = cls % 2 + 3;
  SlabLaunch f = mixed ? pick_slab<float>(spw, xpl) : pick_slab<double>(spw, xpl);
  if (!f) return SNAP_EUNSUPPORTED;
  f(a, st);
  return hipGetLastError() == hipSuccess ? 0 : SNAP_EHIP;
}

}  // namespace snap
