// Newton/SQP projection for implicit 2D diffusion residuals plus one energy
// row per frame (the Navier-Stokes-type constraint set of Appendix A: local
// PDE residuals and a global quadratic invariant per frame), periodic grid.
//
// Rows: r(k, p) = u(p, k+1) - u(p, k) - dt kappa (Lap u)(p, k+1), k < Nt-1,
// and e(t) = sum_p u(p, t)^2 - E_t.  The periodic 5-point Laplacian is
// diagonal in the orthonormal real Fourier basis of a frame (products of
// cos / sin / constant / alternating columns), so in the coordinates
// v_t = Q^T u_t Q (and the residual rows rotated the same way) the problem
// separates into one short time series per Fourier mode w,
//     rows  a_w v(w, k+1) - v(w, k),   a_w = 1 + dt kappa (4/dx^2)(s_j + s_i),
// coupled only through the Nt energy rows sum_w v(w, t)^2 - E_t.  The change
// of coordinates is orthogonal: the objective, the feasible set and the
// projection are the same; u and the residual multipliers are rotated back.
//
// Newton step (Appendix B KKT system, exact Lagrangian Hessian
// W = diag(w_t), w_t = 1 + 2 lambda_E,t per frame), per mode, by null-space
// elimination of the mode's residual rows: their null space is spanned by
// z_t = a^{-t}; a particular solution P of R P = r2 is a weighted prefix sum,
// the reduced Hessian is the scalar sigma = sum_t w_t z_t^2 (positive also
// when some w_t are negative, which happens at the solutions of this family:
// the energy multipliers alternate in sign with magnitudes of 1e2-1e3), and
// the energy rows border the system with the Nt x Nt matrix
//     G = sum_w y_w y_w^T / sigma_w,   y_w,t = 2 v(w, t) z_t,
// accumulated on FP64 MFMA (16 x 16 x 4: one instruction takes four modes).
// The residual multipliers follow from a weighted suffix sum.
//
// Layout: one workgroup of 8 wavefronts per sample.  Spectral arrays are
// mode-major with Nt frames per mode, and lane (t + 16 m) of a wavefront holds
// frame t of the m-th of four consecutive modes (lanes t >= Nt hold zeros and
// touch no memory): a DPP row (16 lanes) is one mode's time series (its prefix
// and suffix sums and reductions are row-local DPP operations), the four rows
// are four modes, and a wavefront's loads are one contiguous run of 4 Nt
// doubles.  Each pass loads the next group of modes before working on the
// current one.
// The frame transforms V = Q^T U Q and U = Q V Q^T are products of N x N
// matrices, done in LDS on FP64 MFMA, 16 x 16 output tiles spread over the
// wavefronts.
//
// Globalization (l1 merit, as the oracle): the exact-W step is taken when it
// exists (every sigma and the border's pivots positive) and passes the
// Armijo test whole or with one second-order correction; otherwise the step
// with W raised to at least 0.1 is used, with the same tests and halving.
// Along any step the residual rows are linear, so ||r(v + a p)||_1 =
// (1 - a) ||r(v)||_1, and the energy rows are quadratic in a with per-frame
// coefficients from two sums: every trial point of the line search costs
// O(Nt) scalar work.
#include "snap_device.hpp"

namespace snap {

namespace {

typedef double dv4 __attribute__((ext_vector_type(4)));

constexpr int kSpT = 16;                  // frames per mode (padded)
constexpr int kSpWaves = 8;
constexpr int kSpThreads = kSpWaves * kWave;
constexpr int kSpMaxN = 64;
constexpr int kSpLd = kSpMaxN + 1;        // LDS row stride of the transform tiles
constexpr double kSpFloor = 0.1;          // Hessian floor of the globalized step
constexpr double kSpLocal = 1e-6;         // local phase: full Newton steps

// per-sample workspace: state header, then five spectral arrays of Nt
// values per mode (mode-major; the residual multipliers' entry Nt-1 stays 0)
struct SpecLayout {
  size_t hdr, vh, v, nu, p, dnu, total;
};

__host__ __device__ inline SpecLayout spec_layout(int n, int nt) {
  const size_t arr = ((size_t)n * n * nt * sizeof(double) + 255) & ~(size_t)255;
  SpecLayout L;
  size_t o = 0;
  L.hdr = o; o += 256;
  L.vh = o; o += arr;
  L.v = o; o += arr;
  L.nu = o; o += arr;
  L.p = o; o += arr;
  L.dnu = o; o += arr;
  L.total = o;
  return L;
}

// basis tables (orthonormal real Fourier basis Q[x][j] and s_j =
// sin^2(pi f_j / N)) for N = 16, 32, 48, 64, packed one after another
__host__ __device__ inline int spec_tab_off(int n) {
  return n == 16 ? 0 : n == 32 ? 272 : n == 48 ? 1328 : 3680;
}

// value of lane `src` (wave-uniform) in every lane
__device__ __forceinline__ double lane_bcast_d(double v, int src) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), src);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), src);
  return __hiloint2double(hi, lo);
}

template <int CTRL>
__device__ __forceinline__ double dpp_bc(double x) {   // out-of-row sources read 0
  return dpp_d<CTRL, 0xf, true>(x);
}
__device__ __forceinline__ double row_next(double x) { return dpp_bc<0x101>(x); }   // lane t+1
__device__ __forceinline__ double row_prev(double x) { return dpp_bc<0x111>(x); }   // lane t-1
// inclusive prefix / suffix sums within each row of 16 lanes
__device__ __forceinline__ double row_prefix(double x) {
  x += dpp_bc<0x111>(x);
  x += dpp_bc<0x112>(x);
  x += dpp_bc<0x114>(x);
  x += dpp_bc<0x118>(x);
  return x;
}
__device__ __forceinline__ double row_suffix(double x) {
  x += dpp_bc<0x101>(x);
  x += dpp_bc<0x102>(x);
  x += dpp_bc<0x104>(x);
  x += dpp_bc<0x108>(x);
  return x;
}
// sum over the row, bit-identical in its 16 lanes (rotations pair the same
// partial sums in swapped order)
__device__ __forceinline__ double row_sum(double x) {
  x += dpp_bc<0x128>(x);
  x += dpp_bc<0x124>(x);
  x += dpp_bc<0x122>(x);
  x += dpp_bc<0x121>(x);
  return x;
}
// sum over the four rows of a wavefront (lanes t, t+16, t+32, t+48)
__device__ __forceinline__ double rows_sum(double x) {
  x += __shfl_xor(x, 16);
  x += __shfl_xor(x, 32);
  return x;
}

// Per-mode elimination of one Newton-type system
//   [[W, R^T, E^T], [R, 0, 0], [E, 0, 0]] [x; dnu; dlE] = [r1; r2; r3]
// restricted to one mode (lane = frame t of that mode): the particular
// solution, z, sigma and x0 (the part of x that does not depend on dlE).
struct ModeSol {
  double z, sig, x0, y;
};

__device__ __forceinline__ ModeSol mode_solve(double r1, double rr2, double v, double w, double a,
                                              int t, int nt) {
  ModeSol m;
  // z = a^-t, az = a^t from the binary digits of t (t < 16)
  const double ra = 1.0 / a;
  const double r2 = ra * ra, r4 = r2 * r2, r8 = r4 * r4;
  const double a2 = a * a, a4 = a2 * a2, a8 = a4 * a4;
  double z = (t & 1) ? ra : 1.0, az = (t & 1) ? a : 1.0;
  z *= (t & 2) ? r2 : 1.0;
  az *= (t & 2) ? a2 : 1.0;
  z *= (t & 4) ? r4 : 1.0;
  az *= (t & 4) ? a4 : 1.0;
  z *= (t & 8) ? r8 : 1.0;
  az *= (t & 8) ? a8 : 1.0;
  const bool valid = t < nt;
  z = valid ? z : 0.0;
  az = valid ? az : 0.0;
  // R P = r2 with P_0 = 0: P_t = a^{-t} sum_{k<t} r2_k a^k
  const double pre = row_prefix(rr2 * az);
  const double P = z * (pre - rr2 * az);
  m.z = z;
  m.sig = row_sum(w * z * z);
  const double c1 = row_sum(z * (r1 - w * P));
  m.x0 = P + z * (c1 / m.sig);
  m.y = 2.0 * v * z;
  return m;
}

// LDS of one workgroup: the transform tiles, or the reductions of the Newton
// passes (never both at once)
struct SpecShared {
  double Q[kSpMaxN * kSpLd];
  union {
    struct {
      double U[kSpMaxN * kSpLd];
      double T[kSpMaxN * kSpLd];
    } tr;
    struct {
      double Gw[kSpWaves][256];          // per-wavefront border partials
      double vec[8][kSpWaves][kSpT];     // per-wavefront per-frame partials
    } nw;
  };
  double s2[kSpMaxN];
  double G[kSpT][kSpT + 1];              // border matrix of the current step
  double Gf[kSpT][kSpT + 1], rf[kSpT], xs[kSpT];   // its elimination
  double lE[kSpT], dlE[kSpT], lq[kSpT];  // energy multipliers, step, correction
  double wt[kSpT];                       // W per frame of the current step
  double hE[kSpT], A[kSpT], B[kSpT], bv[kSpT];
  double tot[8][kSpT];                   // workgroup totals of the per-frame slots
  double h1res, scal[8];
  double red[kSpWaves][8];
  int flag[8];
};

// ---------------------------------------------------------------- transforms
// 16 x 16 tile of C = A B over K (a multiple of 4) on FP64 MFMA; A and B are
// read through accessors (row, col).  Result element e of lane (j + 16 g) is
// C[g + 4e][j].
template <class FA, class FB>
__device__ __forceinline__ dv4 tile_mm(int K, FA fa, FB fb) {
  const int lane = threadIdx.x & (kWave - 1);
  const int li = lane & 15, lk = lane >> 4;
  dv4 acc = {0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < K; k0 += 4)
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(fa(li, k0 + lk), fb(k0 + lk, li), acc, 0, 0, 0);
  return acc;
}

// physical frame src[y*N + x] -> spectral column t of the mode-major arrays
// dst (and dst2 if not null): V = Q^T U Q
__device__ void frame_forward(SpecShared& sh, int n, int nt, const double* src, double* dst,
                              double* dst2, int t, double* umax) {
  const int tid = threadIdx.x, wv = tid / kWave, lane = tid & (kWave - 1);
  const int li = lane & 15, lk = lane >> 4;
  double mx = 0.0;
  for (int e = tid; e < n * n; e += kSpThreads) {
    const double x = src[e];
    sh.tr.U[(e / n) * kSpLd + (e % n)] = x;
    // fmax drops NaN: a non-finite value is carried as +inf
    mx = fmax(mx, finite(x) ? fabs(x) : __builtin_inf());
  }
  if (umax) *umax = fmax(*umax, mx);
  __syncthreads();
  const int nb = n / 16;
  for (int tl = wv; tl < nb * nb; tl += kSpWaves) {   // T = U Q
    const int y0 = (tl / nb) * 16, i0 = (tl % nb) * 16;
    const dv4 c = tile_mm(n, [&](int i, int k) { return sh.tr.U[(y0 + i) * kSpLd + k]; },
                          [&](int k, int j) { return sh.Q[k * kSpLd + i0 + j]; });
#pragma unroll
    for (int e = 0; e < 4; ++e) sh.tr.T[(y0 + lk + 4 * e) * kSpLd + i0 + li] = c[e];
  }
  __syncthreads();
  for (int tl = wv; tl < nb * nb; tl += kSpWaves) {   // V = Q^T T
    const int j0 = (tl / nb) * 16, i0 = (tl % nb) * 16;
    const dv4 c = tile_mm(n, [&](int i, int k) { return sh.Q[k * kSpLd + j0 + i]; },
                          [&](int k, int j) { return sh.tr.T[k * kSpLd + i0 + j]; });
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const size_t w = (size_t)(j0 + lk + 4 * e) * n + i0 + li;
      dst[w * nt + t] = c[e];
      if (dst2) dst2[w * nt + t] = c[e];
    }
  }
  __syncthreads();
}

// spectral column t of the mode-major array src -> physical frame dst: U = Q V Q^T
__device__ void frame_inverse(SpecShared& sh, int n, int nt, const double* src, int t, double* dst) {
  const int tid = threadIdx.x, wv = tid / kWave, lane = tid & (kWave - 1);
  const int li = lane & 15, lk = lane >> 4;
  for (int e = tid; e < n * n; e += kSpThreads) sh.tr.U[(e / n) * kSpLd + (e % n)] = src[(size_t)e * nt + t];
  __syncthreads();
  const int nb = n / 16;
  for (int tl = wv; tl < nb * nb; tl += kSpWaves) {   // T = V Q^T
    const int j0 = (tl / nb) * 16, x0 = (tl % nb) * 16;
    const dv4 c = tile_mm(n, [&](int i, int k) { return sh.tr.U[(j0 + i) * kSpLd + k]; },
                          [&](int k, int j) { return sh.Q[(x0 + j) * kSpLd + k]; });
#pragma unroll
    for (int e = 0; e < 4; ++e) sh.tr.T[(j0 + lk + 4 * e) * kSpLd + x0 + li] = c[e];
  }
  __syncthreads();
  for (int tl = wv; tl < nb * nb; tl += kSpWaves) {   // U = Q T
    const int y0 = (tl / nb) * 16, x0 = (tl % nb) * 16;
    const dv4 c = tile_mm(n, [&](int i, int k) { return sh.Q[(y0 + i) * kSpLd + k]; },
                          [&](int k, int j) { return sh.tr.T[k * kSpLd + x0 + j]; });
#pragma unroll
    for (int e = 0; e < 4; ++e) dst[(y0 + lk + 4 * e) * n + x0 + li] = c[e];
  }
  __syncthreads();
}

// ---------------------------------------------------------------- reductions
// per-frame partial (lane t of every row) into slot `s`, summed over the
// wavefront's four rows; the workgroup total is formed by spec_frames
__device__ __forceinline__ void put_frames(SpecShared& sh, int s, double x) {
  x = rows_sum(x);
  const int lane = threadIdx.x & (kWave - 1);
  if (lane < kSpT) sh.nw.vec[s][threadIdx.x / kWave][lane] = x;
}
// workgroup totals of per-frame slots [first, first + count) into sh.tot
// (one thread per slot and frame; a barrier must follow)
__device__ __forceinline__ void total_frames(SpecShared& sh, int first, int count) {
  const int idx = threadIdx.x;
  if (idx < count * kSpT) {
    const int s = first + idx / kSpT, t = idx % kSpT;
    double acc = 0.0;
    for (int q = 0; q < kSpWaves; ++q) acc += sh.nw.vec[s][q][t];
    sh.tot[s][t] = acc;
  }
}
// scalar partials (sum or max of non-negative values) per wavefront
__device__ __forceinline__ void put_scalar(SpecShared& sh, int s, double x, bool is_max) {
  x = is_max ? wave_max(x) : wave_sum(x);
  if ((threadIdx.x & (kWave - 1)) == 0) sh.red[threadIdx.x / kWave][s] = x;
}
__device__ __forceinline__ double scalar_total(const SpecShared& sh, int s, bool is_max) {
  double acc = 0.0;
  for (int q = 0; q < kSpWaves; ++q) acc = is_max ? fmax(acc, sh.red[q][s]) : acc + sh.red[q][s];
  return acc;
}

// Solve G x = b (nt x nt, symmetric; frames past nt are identity rows) by
// elimination without pivoting in wavefront 0 on an LDS copy, lane i
// updating row i; back substitution by lane 0.  Returns false if a pivot is
// not positive.  x is written to out[0..16).
__device__ bool border_solve(SpecShared& sh, const double* b, double* out, int nt) {
  const int lane = threadIdx.x & (kWave - 1);
  const int i = lane & 15;
  const bool own = lane < kSpT;
  if (own) {
    for (int j = 0; j < kSpT; ++j) sh.Gf[i][j] = (i < nt && j < nt) ? sh.G[i][j] : (i == j ? 1.0 : 0.0);
    sh.rf[i] = i < nt ? b[i] : 0.0;
  }
  wave_sync();
  bool ok = true;
  for (int p = 0; p < kSpT; ++p) {
    const double dp = sh.Gf[p][p];
    ok = ok && dp > 0.0;
    if (own && i > p) {
      const double l = sh.Gf[i][p] / dp;
      for (int j = p + 1; j < kSpT; ++j) sh.Gf[i][j] -= l * sh.Gf[p][j];
      sh.rf[i] -= l * sh.rf[p];
    }
    wave_sync();
  }
  if (lane == 0) {
    for (int p = kSpT - 1; p >= 0; --p) {
      double x = sh.rf[p];
      for (int j = p + 1; j < kSpT; ++j) x -= sh.Gf[p][j] * sh.xs[j];
      x /= sh.Gf[p][p];
      sh.xs[p] = x;
      out[p] = p < nt ? x : 0.0;
    }
  }
  wave_sync();
  return ok;
}

// state of one sample kept in its workspace header between launches is not
// needed: the whole Newton loop runs in one launch
struct SpecCtx {
  int n, nt, modes;
  double coef;                 // dt kappa 4 / dx^2
  double s_phys;               // dt kappa / dx^2
  const double* uh;            // u_hat (forward) / u* (adjoint) physical
  double *vh, *v, *nu, *p, *dnu;
};

__device__ __forceinline__ double mode_a(const SpecShared& sh, const SpecCtx& C, int w) {
  const int j = w / C.n, i = w - j * C.n;
  return 1.0 + C.coef * (sh.s2[j] + sh.s2[i]);
}

// value of frame t of mode (4 grp + km) in a spectral array (0 past Nt, with
// no memory access)
__device__ __forceinline__ double sld(const double* a, const SpecCtx& C, int grp, int km, int t) {
  return t < C.nt ? a[(size_t)(4 * grp + km) * C.nt + t] : 0.0;
}

// Pass A: residuals and stationarity at (v, nu, lE) (forward) or the adjoint
// right-hand side (bwd), and the elimination with W = sh.wt: border G, its
// right-hand side b, convergence measures.  Per-frame slots: 0 b, 1 sum v^2,
// 2 sum |r| (rows k), 3 sum r^2, 4 sum g^2; scalar slot 0: min sigma.
__device__ void pass_assemble(SpecShared& sh, const SpecCtx& C, bool bwd) {
  const int tid = threadIdx.x, wv = tid / kWave, lane = tid & (kWave - 1);
  const int t = lane & 15, km = lane >> 4;
  const bool valid = t < C.nt, rowk = t + 1 < C.nt;
  const double w = sh.wt[t], lE = valid ? sh.lE[t] : 0.0;
  const int ng = C.modes / 4;
  dv4 gacc = {0.0, 0.0, 0.0, 0.0};
  double bacc = 0.0, e2 = 0.0, h1 = 0.0, h2 = 0.0, g2 = 0.0, smin = 1e300;
  double vn_ = 0.0, vhn_ = 0.0, nun_ = 0.0;   // the next group, loaded ahead
  if (wv < ng) {
    vn_ = sld(C.v, C, wv, km, t);
    vhn_ = sld(C.vh, C, wv, km, t);
    if (!bwd) nun_ = sld(C.nu, C, wv, km, t);
  }
#pragma unroll 1
  for (int grp = wv; grp < ng; grp += kSpWaves) {
    const double v = vn_, vh = vhn_, nu = nun_;
    if (grp + kSpWaves < ng) {
      vn_ = sld(C.v, C, grp + kSpWaves, km, t);
      vhn_ = sld(C.vh, C, grp + kSpWaves, km, t);
      if (!bwd) nun_ = sld(C.nu, C, grp + kSpWaves, km, t);
    }
    const double a = mode_a(sh, C, 4 * grp + km);
    // cross-lane reads outside any branch: a lane that is switched off
    // would hand its neighbours 0
    const double vnext = row_next(v);
    const double nprev = row_prev(nu);
    double r1, r2;
    if (!bwd) {
      const double hk = rowk ? a * vnext - v : 0.0;
      const double g = valid ? v - vh - (rowk ? nu : 0.0) + (t >= 1 ? a * nprev : 0.0) + 2.0 * v * lE : 0.0;
      r1 = -g;
      r2 = -hk;
      h1 += fabs(hk);
      h2 += hk * hk;
      g2 += g * g;
      e2 += v * v;
    } else {
      r1 = vh;   // the upstream gradient, rotated
      r2 = 0.0;
    }
    const ModeSol ms = mode_solve(r1, r2, v, w, a, t, C.nt);
    smin = fmin(smin, ms.sig);
    const double ys = ms.y / ms.sig;
    gacc = __builtin_amdgcn_mfma_f64_16x16x4f64(ms.y, ys, gacc, 0, 0, 0);
    bacc += 2.0 * v * ms.x0;
  }
#pragma unroll
  for (int e = 0; e < 4; ++e) sh.nw.Gw[wv][(km + 4 * e) * 16 + t] = gacc[e];
  put_frames(sh, 0, bacc);
  put_frames(sh, 1, e2);
  put_frames(sh, 2, h1);
  put_frames(sh, 3, h2);
  put_frames(sh, 4, g2);
  smin = fmin(smin, __shfl_xor(smin, 16));
  smin = fmin(smin, __shfl_xor(smin, 32));
  double sm = smin;
#pragma unroll
  for (int off = 8; off >= 1; off >>= 1) sm = fmin(sm, __shfl_xor(sm, off));
  if (lane == 0) sh.red[wv][0] = sm;
  __syncthreads();
  if (tid < 256) {
    double acc = 0.0;
    for (int q = 0; q < kSpWaves; ++q) acc += sh.nw.Gw[q][tid];
    sh.G[tid >> 4][tid & 15] = acc;
  }
  total_frames(sh, 0, 5);
  __syncthreads();
}

// Pass B: the step x = x0 - z (y . dlE) / sigma and the residual-multiplier
// step from R^T dnu = r1 - E dlE - W x (suffix sums), written to p / dnu,
// with the merit sums.  Per-frame slots: 0 sum v x, 1 sum x^2; scalar slots:
// 1 sum (v - v_hat) x, 2 sum x^2, 3 max |nu + dnu|.  The adjoint writes x only.
__device__ void pass_step(SpecShared& sh, const SpecCtx& C, bool bwd) {
  const int tid = threadIdx.x, wv = tid / kWave, lane = tid & (kWave - 1);
  const int t = lane & 15, km = lane >> 4;
  const bool valid = t < C.nt, rowk = t + 1 < C.nt;
  const double w = sh.wt[t], lE = valid ? sh.lE[t] : 0.0, dl = valid ? sh.dlE[t] : 0.0;
  const int ng = C.modes / 4;
  double fa = 0.0, fb = 0.0, dp = 0.0, pp = 0.0, lmax = 0.0;
  double vn_ = 0.0, vhn_ = 0.0, nun_ = 0.0;
  if (wv < ng) {
    vn_ = sld(C.v, C, wv, km, t);
    vhn_ = sld(C.vh, C, wv, km, t);
    if (!bwd) nun_ = sld(C.nu, C, wv, km, t);
  }
#pragma unroll 1
  for (int grp = wv; grp < ng; grp += kSpWaves) {
    const double v = vn_, vh = vhn_, nu = nun_;
    if (grp + kSpWaves < ng) {
      vn_ = sld(C.v, C, grp + kSpWaves, km, t);
      vhn_ = sld(C.vh, C, grp + kSpWaves, km, t);
      if (!bwd) nun_ = sld(C.nu, C, grp + kSpWaves, km, t);
    }
    const size_t o = (size_t)(4 * grp + km) * C.nt + t;
    const double a = mode_a(sh, C, 4 * grp + km);
    const double vnext = row_next(v);
    const double nprev = row_prev(nu);
    double r1, r2;
    if (!bwd) {
      const double hk = rowk ? a * vnext - v : 0.0;
      const double g = valid ? v - vh - (rowk ? nu : 0.0) + (t >= 1 ? a * nprev : 0.0) + 2.0 * v * lE : 0.0;
      r1 = -g;
      r2 = -hk;
    } else {
      r1 = vh;
      r2 = 0.0;
    }
    const ModeSol ms = mode_solve(r1, r2, v, w, a, t, C.nt);
    const double x = ms.x0 - ms.z * (row_sum(ms.y * dl) / ms.sig);
    if (valid) C.p[o] = x;
    if (bwd) continue;
    // R^T dnu = q, q = r1 - E dlE - W x: dnu_t = (sum_{s>t} q_s z_s) / z_t
    const double q = valid ? r1 - 2.0 * v * dl - w * x : 0.0;
    const double qz = q * ms.z;
    const double suf = row_suffix(qz) - qz;
    const double dn = rowk ? suf / ms.z : 0.0;
    if (valid) C.dnu[o] = dn;
    const double d = v - vh;
    fa += v * x;
    fb += x * x;
    dp += d * x;
    pp += x * x;
    lmax = fmax(lmax, fabs(nu + dn));
  }
  if (!bwd) {
    put_frames(sh, 0, fa);
    put_frames(sh, 1, fb);
    put_scalar(sh, 1, dp, false);
    put_scalar(sh, 2, pp, false);
    put_scalar(sh, 3, lmax, true);
  }
  __syncthreads();
  if (!bwd) {
    total_frames(sh, 0, 2);
    __syncthreads();
  }
}

// Pass C: the second-order correction q = -z (y . lq) / sigma (a vector of
// the residual rows' null space: it changes only the energy rows) and its
// merit sums.  Per-frame slots: 2 sum (v + p) q, 3 sum q^2; scalar slots:
// 4 sum (v - v_hat) q, 5 sum p q, 6 sum q^2.
__device__ void pass_correction(SpecShared& sh, const SpecCtx& C) {
  const int tid = threadIdx.x, wv = tid / kWave, lane = tid & (kWave - 1);
  const int t = lane & 15, km = lane >> 4;
  const double w = sh.wt[t], lq = t < C.nt ? sh.lq[t] : 0.0;
  const int ng = C.modes / 4;
  double fc = 0.0, fd = 0.0, dq = 0.0, pq = 0.0, qq = 0.0;
  double vn_ = 0.0, vhn_ = 0.0, xn_ = 0.0;
  if (wv < ng) {
    vn_ = sld(C.v, C, wv, km, t);
    vhn_ = sld(C.vh, C, wv, km, t);
    xn_ = sld(C.p, C, wv, km, t);
  }
#pragma unroll 1
  for (int grp = wv; grp < ng; grp += kSpWaves) {
    const double v = vn_, vh = vhn_, x = xn_;
    if (grp + kSpWaves < ng) {
      vn_ = sld(C.v, C, grp + kSpWaves, km, t);
      vhn_ = sld(C.vh, C, grp + kSpWaves, km, t);
      xn_ = sld(C.p, C, grp + kSpWaves, km, t);
    }
    const double a = mode_a(sh, C, 4 * grp + km);
    const ModeSol ms = mode_solve(0.0, 0.0, v, w, a, t, C.nt);
    const double q = -ms.z * (row_sum(ms.y * lq) / ms.sig);
    fc += (v + x) * q;
    fd += q * q;
    dq += (v - vh) * q;
    pq += x * q;
    qq += q * q;
  }
  put_frames(sh, 2, fc);
  put_frames(sh, 3, fd);
  put_scalar(sh, 4, dq, false);
  put_scalar(sh, 5, pq, false);
  put_scalar(sh, 6, qq, false);
  __syncthreads();
  total_frames(sh, 2, 2);
  __syncthreads();
}

// Pass U: v += alpha (p [+ q]), nu += alpha dnu
__device__ void pass_update(SpecShared& sh, const SpecCtx& C, double alpha, bool soc) {
  const int tid = threadIdx.x, wv = tid / kWave, lane = tid & (kWave - 1);
  const int t = lane & 15, km = lane >> 4;
  const bool valid = t < C.nt;
  const double w = sh.wt[t], lq = valid ? sh.lq[t] : 0.0;
  const int ng = C.modes / 4;
#pragma unroll 1
  for (int grp = wv; grp < ng; grp += kSpWaves) {
    const size_t o = (size_t)(4 * grp + km) * C.nt + t;
    const double v = sld(C.v, C, grp, km, t);
    const double x = sld(C.p, C, grp, km, t);
    const double nu = sld(C.nu, C, grp, km, t);
    const double dn = sld(C.dnu, C, grp, km, t);
    double step = x;
    if (soc) {
      const double a = mode_a(sh, C, 4 * grp + km);
      const ModeSol ms = mode_solve(0.0, 0.0, v, w, a, t, C.nt);
      step += -ms.z * (row_sum(ms.y * lq) / ms.sig);
    }
    if (valid) {
      C.v[o] = v + alpha * step;
      C.nu[o] = nu + alpha * dn;
    }
  }
  __syncthreads();
}

}  // namespace

// one workgroup per sample: the whole Newton loop, transforms included
__global__ __launch_bounds__(kSpThreads, 1) void spec_kernel(KernelArgs A) {
  const int sid = A.order[blockIdx.x];
  const snap_sample_desc D = A.descs[sid];
  __shared__ SpecShared sh;
  const int tid = threadIdx.x;
  const int n = D.nx, nt = D.nt, np = n * n;
  const bool bwd = A.backward != 0;
  const SpecLayout L = spec_layout(n, nt);
  unsigned char* ws = A.ws + A.ws_off[sid];
  SpecCtx C;
  C.n = n; C.nt = nt; C.modes = np;
  C.s_phys = D.dt * D.p0 / (D.dx * D.dx);
  C.coef = 4.0 * C.s_phys;
  C.vh = (double*)(ws + L.vh); C.v = (double*)(ws + L.v); C.nu = (double*)(ws + L.nu);
  C.p = (double*)(ws + L.p); C.dnu = (double*)(ws + L.dnu);
  const double* tab = A.tab + spec_tab_off(n);
  double* uo = A.u + D.var_off;
  double* lam = A.lam + D.row_off;
  const double* E = A.aux + D.aux_off;
  const int mres = (nt - 1) * np;

  for (int e = tid; e < np; e += kSpThreads) sh.Q[(e / n) * kSpLd + (e % n)] = tab[e];
  for (int e = tid; e < n; e += kSpThreads) sh.s2[e] = tab[np + e];
  __syncthreads();

  if (bwd) {
    // adjoint: (u*, lam*) rotated; the upstream gradient rotated into vh
    for (int t = 0; t < nt; ++t) {
      frame_forward(sh, n, nt, uo + (size_t)t * np, C.v, nullptr, t, nullptr);
      frame_forward(sh, n, nt, A.grad_u + D.var_off + (size_t)t * np, C.vh, nullptr, t, nullptr);
    }
    if (tid < kSpT) {
      sh.lE[tid] = tid < nt ? lam[mres + tid] : 0.0;
      sh.wt[tid] = tid < nt ? 1.0 + 2.0 * sh.lE[tid] : 1.0;
    }
    __syncthreads();
    pass_assemble(sh, C, true);
    bool ok = true;
    if (tid < kSpT) sh.bv[tid] = tid < nt ? sh.tot[0][tid] : 0.0;
    __syncthreads();
    if (tid < kWave) {
      ok = border_solve(sh, sh.bv, sh.dlE, nt);
      if (tid == 0) sh.flag[0] = ok ? 1 : 0;
    }
    __syncthreads();
    // min sigma over the wavefronts (slot 0 holds minima)
    if (tid == 0) {
      double sm = 1e300;
      for (int q = 0; q < kSpWaves; ++q) sm = fmin(sm, sh.red[q][0]);
      if (!(sm > 0.0)) sh.flag[0] = 0;
    }
    __syncthreads();
    const bool good = sh.flag[0] != 0;
    pass_step(sh, C, true);
    for (int t = 0; t < nt; ++t) frame_inverse(sh, n, nt, C.p, t, A.grad_uhat + D.var_off + (size_t)t * np);
    if (tid == 0) {
      snap_sample_stats st;
      st.status = good ? SNAP_ST_CONVERGED : SNAP_ST_SINGULAR_PIVOT;
      st.newton_iters = 0; st.ls_backtracks = 0; st.refine_steps = 0;
      st.h_inf = 0.0; st.stat_inf = 0.0;
      A.stats[sid] = st;
    }
    return;
  }

  // forward: v_hat = v = rotated u_hat, nu = 0, lE = 0
  double umax = 0.0;
  for (int t = 0; t < nt; ++t)
    frame_forward(sh, n, nt, A.uhat + D.var_off + (size_t)t * np, C.vh, C.v, t, &umax);
  for (int e = tid; e < np * nt; e += kSpThreads) C.nu[e] = 0.0;
  {
    const double um = wave_max(umax);
    if ((tid & (kWave - 1)) == 0) sh.red[tid / kWave][7] = um;
  }
  if (tid < kSpT) { sh.lE[tid] = 0.0; sh.dlE[tid] = 0.0; sh.lq[tid] = 0.0; }
  __syncthreads();
  const double uscale = 1.0 + scalar_total(sh, 7, true);
  const bool input_ok = finite(uscale);

  double mu = 0.0;
  int iters = 0, backtracks = 0, status = SNAP_ST_MAX_ITER;
  for (int it = 0;; ++it) {
    // exact Hessian of the Lagrangian, and whether the floor changes it
    if (tid < kSpT) sh.wt[tid] = tid < nt ? 1.0 + 2.0 * sh.lE[tid] : 1.0;
    __syncthreads();
    pass_assemble(sh, C, false);
    // wavefront 0: convergence test, border solve of the exact step
    if (tid < kWave) {
      const int lane = tid;
      double hE = 0.0, hr2 = 0.0, g2 = 0.0, h1r = 0.0, bt = 0.0;
      if (lane < kSpT && lane < nt) {
        hE = sh.tot[1][lane] - E[lane];
        hr2 = sh.tot[3][lane];
        g2 = sh.tot[4][lane];
        h1r = sh.tot[2][lane];
        bt = sh.tot[0][lane] + hE;
      }
      // per-frame 2-norms bound the physical max-norms (the rotation is orthogonal)
      const double hinf = fmax(wave_max(fabs(hE)), sqrt(wave_max(hr2)));
      const double sinf = sqrt(wave_max(g2));
      // (wave_max's fmax drops NaN: the sums are tested for finiteness too)
      const bool nonfin = __any(!finite(hE) || !finite(hr2) || !finite(g2)) || !input_ok;
      const double h1 = wave_sum(fabs(hE)) + wave_sum(h1r);
      double sm = 1e300;
      for (int q = 0; q < kSpWaves; ++q) sm = fmin(sm, sh.red[q][0]);
      if (lane < kSpT) { sh.hE[lane] = hE; sh.bv[lane] = bt; }
      wave_sync();
      int done = 0;
      if (nonfin || !finite(hinf) || !finite(sinf)) done = 2;
      else if (hinf <= A.opt.tol_h && sinf <= A.opt.tol_s * uscale) done = 1;
      else if (it >= A.opt.max_newton) done = 3;
      bool ok = false;
      if (!done) ok = border_solve(sh, sh.bv, sh.dlE, nt) && sm > 0.0;
      if (lane == 0) {
        sh.flag[0] = done;
        sh.flag[1] = ok ? 1 : 0;
        sh.scal[0] = hinf; sh.scal[1] = sinf; sh.scal[2] = h1;
        sh.h1res = wave_sum(h1r);
      }
    }
    __syncthreads();
    const int done = sh.flag[0];
    if (done) {
      status = done == 1 ? SNAP_ST_CONVERGED : (done == 2 ? SNAP_ST_NONFINITE : SNAP_ST_MAX_ITER);
      break;
    }
    const double hinf = sh.scal[0], h1 = sh.scal[2], h1r = sh.h1res;
    const bool local = hinf <= kSpLocal;
    // scalar line search on the energy rows' per-frame quadratics
    auto dphi_at = [&](double alpha, double muv, double dp, double pp) {
      double e1 = 0.0;
      for (int t = 0; t < nt; ++t) e1 += fabs(sh.hE[t] + 2.0 * alpha * sh.A[t] + alpha * alpha * sh.B[t]);
      return alpha * dp + 0.5 * alpha * alpha * pp + muv * (e1 + (1.0 - alpha) * h1r - h1);
    };
    // tests of the step in p (thread 0): full step, or a correction to try
    auto decide = [&]() {
      if (tid == 0) {
        for (int t = 0; t < kSpT; ++t) {
          sh.A[t] = t < nt ? sh.tot[0][t] : 0.0;
          sh.B[t] = t < nt ? sh.tot[1][t] : 0.0;
        }
        const double dp = scalar_total(sh, 1, false), pp = scalar_total(sh, 2, false);
        double lm = scalar_total(sh, 3, true);
        for (int t = 0; t < nt; ++t) lm = fmax(lm, fabs(sh.lE[t] + sh.dlE[t]));
        const double mut = fmax(mu, 1.1 * lm + 1e-8);
        const double Dd = dp - mut * h1;
        int acc = 0, try_soc = 0;
        if (local) acc = 1;
        else if (Dd < 0.0) {
          if (dphi_at(1.0, mut, dp, pp) <= 1e-4 * Dd) acc = 1;
          else try_soc = 1;
        }
        sh.scal[3] = mut; sh.scal[4] = Dd; sh.scal[5] = dp; sh.scal[6] = pp;
        sh.flag[3] = acc; sh.flag[4] = try_soc;
      }
      __syncthreads();
      if (sh.flag[4]) {
        // one second-order correction: G lq = h_E(v + p) with the same border
        if (tid < kSpT) sh.bv[tid] = tid < nt ? sh.hE[tid] + 2.0 * sh.A[tid] + sh.B[tid] : 0.0;
        __syncthreads();
        if (tid < kWave) (void)border_solve(sh, sh.bv, sh.lq, nt);
        __syncthreads();
        pass_correction(sh, C);
        if (tid == 0) {
          const double mut = sh.scal[3], Dd = sh.scal[4], dp = sh.scal[5], pp = sh.scal[6];
          const double dq = scalar_total(sh, 4, false), pq = scalar_total(sh, 5, false),
                       qq = scalar_total(sh, 6, false);
          double e1 = 0.0;
          for (int t = 0; t < nt; ++t)
            e1 += fabs(sh.hE[t] + 2.0 * sh.A[t] + sh.B[t] + 2.0 * sh.tot[2][t] +
                       sh.tot[3][t]);
          // residual rows: r(v + p + q) = 0 (p solves them, q is in their null space)
          const double ds = dp + dq + 0.5 * (pp + 2.0 * pq + qq) + mut * (e1 - h1);
          sh.flag[3] = ds <= 1e-4 * Dd ? 2 : 0;
        }
        __syncthreads();
      }
      return sh.flag[3];
    };
    int accepted = 0;        // 1 step, 2 step + correction
    double alpha = 1.0;
    bool have = sh.flag[1] != 0;   // the exact-W elimination exists
    if (have) {
      pass_step(sh, C, false);
      accepted = decide();
    }
    if (!accepted) {
      const int raised = __syncthreads_or(tid < nt && sh.wt[tid] < kSpFloor);
      if (raised || !have) {
        // the step with W raised to the floor
        if (tid < kSpT) sh.wt[tid] = fmax(sh.wt[tid], kSpFloor);
        __syncthreads();
        pass_assemble(sh, C, false);
        if (tid < kSpT) sh.bv[tid] = tid < nt ? sh.tot[0][tid] + sh.hE[tid] : 0.0;
        __syncthreads();
        if (tid < kWave) {
          const bool ok = border_solve(sh, sh.bv, sh.dlE, nt);
          if (tid == 0) sh.flag[1] = ok ? 1 : 0;
        }
        __syncthreads();
        have = sh.flag[1] != 0;
        if (have) {
          pass_step(sh, C, false);
          accepted = decide();
        }
      }
      if (!accepted && have) {
        // halving along the step in p
        if (tid == 0) {
          const double mut = sh.scal[3], Dd = sh.scal[4], dp = sh.scal[5], pp = sh.scal[6];
          double al = 1.0;
          int ok = 0, nb = 0;
          if (Dd < 0.0) {
            for (int ls = 0; ls < A.opt.max_ls; ++ls) {
              al *= 0.5;
              ++nb;
              if (dphi_at(al, mut, dp, pp) <= 1e-4 * al * Dd) { ok = 1; break; }
            }
          }
          sh.flag[3] = ok;
          sh.scal[7] = al;
          sh.flag[5] = nb;
        }
        __syncthreads();
        backtracks += sh.flag[5];
        if (sh.flag[3]) { accepted = 1; alpha = sh.scal[7]; }
      }
    }
    if (accepted) mu = sh.scal[3];
    if (!accepted) {
      status = SNAP_ST_LS_FAIL;
      __syncthreads();
      break;
    }
    pass_update(sh, C, alpha, accepted == 2);
    if (tid < kSpT) sh.lE[tid] += alpha * sh.dlE[tid];
    ++iters;
    __syncthreads();
  }

  // outputs: u and the residual multipliers rotated back, energy multipliers
  for (int t = 0; t < nt; ++t) frame_inverse(sh, n, nt, C.v, t, uo + (size_t)t * np);
  for (int k = 0; k + 1 < nt; ++k) frame_inverse(sh, n, nt, C.nu, k, lam + (size_t)k * np);
  if (tid < nt) lam[mres + tid] = sh.lE[tid];
  __syncthreads();
  // statistics of the physical rows at the returned point
  const double s = C.s_phys;
  const double* uh = A.uhat + D.var_off;
  double hm = 0.0, sm = 0.0;
  for (int e = tid; e < nt * np; e += kSpThreads) {
    const int t = e / np, pidx = e - t * np, y = pidx / n, x = pidx - y * n;
    const int xm = x == 0 ? n - 1 : x - 1, xp = x == n - 1 ? 0 : x + 1;
    const int ym = y == 0 ? n - 1 : y - 1, yp = y == n - 1 ? 0 : y + 1;
    auto nb4 = [&](const double* f) {
      return f[ym * n + x] + f[yp * n + x] + f[y * n + xm] + f[y * n + xp];
    };
    const double* ut = uo + (size_t)t * np;
    const double uu = ut[pidx];
    double st = uu - uh[e] + 2.0 * uu * lam[mres + t];
    if (t + 1 < nt) {
      const double* un = ut + np;
      const double r = un[pidx] * (1.0 + 4.0 * s) - s * nb4(un) - uu;
      hm = fmax(hm, fabs(r));
      st -= lam[(size_t)t * np + pidx];
    }
    if (t >= 1) {
      const double* lp = lam + (size_t)(t - 1) * np;
      st += lp[pidx] * (1.0 + 4.0 * s) - s * nb4(lp);
    }
    sm = fmax(sm, fabs(st));
    if (!finite(st)) sm = __builtin_nan("");
  }
  put_scalar(sh, 0, hm, true);
  put_scalar(sh, 1, sm, true);
  // energy rows
  for (int t = 0; t < nt; ++t) {
    double e2 = 0.0;
    for (int e = tid; e < np; e += kSpThreads) {
      const double uu = uo[(size_t)t * np + e];
      e2 += uu * uu;
    }
    e2 = wave_sum(e2);
    if ((tid & (kWave - 1)) == 0) sh.nw.vec[0][tid / kWave][t] = e2;
  }
  __syncthreads();
  total_frames(sh, 0, 1);
  __syncthreads();
  if (tid == 0) {
    double hmax = scalar_total(sh, 0, true);
    for (int t = 0; t < nt; ++t) hmax = fmax(hmax, fabs(sh.tot[0][t] - E[t]));
    snap_sample_stats st;
    st.status = status;
    st.newton_iters = iters;
    st.ls_backtracks = backtracks;
    st.refine_steps = 0;
    st.h_inf = hmax;
    st.stat_inf = scalar_total(sh, 1, true);
    A.stats[sid] = st;
  }
}

bool spec_supported(int nx, int ny, int nt) {
  return nx == ny && (nx == 16 || nx == 32 || nx == 48 || nx == 64) && nt >= 1 && nt <= kSpT;
}

size_t spec_workspace_bytes(int nx, int nt) { return spec_layout(nx, nt).total; }

int spec_launch(const KernelArgs& a, hipStream_t st) {
  if (a.count == 0) return 0;
  hipLaunchKernelGGL(spec_kernel, dim3(a.count), dim3(kSpThreads), 0, st, a);
  return hipGetLastError() == hipSuccess ? 0 : SNAP_EHIP;
}

}  // namespace snap
