// Newton/SQP projection for local flux-residual constraints (viscous Burgers,
// Lax-Friedrichs flux, periodic x): the banded Schur-complement path.
//
// Rows (k, x), k = 0..Nt-2, involve u(x, k+1) and u(x-1..x+1, k) (paper
// Appendix D flux residual; Sec. III-B: local couplings give a sparse, here
// banded, Jacobian).  With W = I + Hess(lam^T h) (diagonal: the flux is
// separable), the Newton-KKT system of Appendix B reduces to
//     S lam+ = h - J W^{-1}(u - u_hat),   S = J W^{-1} J^T,
//     p = -W^{-1}(u - u_hat + J^T lam+).
// S is symmetric positive definite and, with rows ordered slab-major and
// "folded" inside a slab (x = 0, Nx-1, 1, Nx-2, ...: periodic neighbours end up
// at most two positions apart), banded with half-bandwidth b = Nx + 2.
//
// Factorization: S = L D L^T by a right-looking block-band LDL^T with 16x16
// blocks (block half-bandwidth BB = ceil(b/16)).  One workgroup per sample.
// The live window (block rows J..J+BB) lives in MFMA accumulator registers:
// block (I, I-d) is kept in slot (d, I mod (BB+1-d)), a fixed owner, so a
// retiring panel block is replaced in place by the entering block of row
// J+BB+1.  Per panel J:
//   1. the diagonal block is factored in registers by one wavefront (lane k
//      holds column k, lane 16 + k column k of the identity; pivot columns are
//      broadcast lane to lane and both apply the same row operations), giving
//      D_J, L_JJ^{-1}, T = L_JJ^{-T} D_J^{-1} and the forward-substitution block;
//   2. panel blocks L(I,J) = S(I,J) T   (MFMA);
//   3. trailing update S(I,K) -= L(I,J) D_J L(K,J)^T   (MFMA, rank 16);
//   4. the entering block row is assembled from the stencil (S is never
//      stored unfactored) and the forward substitution L y = r advances.
// The factor (L_JJ^{-1}, L(I,J), D) is written to the workspace for the
// backward substitution and for the adjoint.
//
// Long wide bands are factored in a two-sided form: two workgroups per sample
// factor the band from both ends toward a separator of BB block rows, which a
// third sweep factors last (the parts section below).  With the option flag
// SNAP_FLAG_SOC a rejected full step gets one second-order correction
// (band_soc) before halving.
//
// Precision R: double (plain form) or float (mixed form: float32 factor and
// solves, float64 residual r - S x from the stencil, iterative refinement).
#include <type_traits>

#include "snap_device.hpp"

namespace snap {

typedef double dvec4 __attribute__((ext_vector_type(4)));
typedef float fvec4 __attribute__((ext_vector_type(4)));

template <typename R> struct Mfma;
// Operand layouts (both types): A[i][k] in lane i + 16k, B[k][j] in lane j + 16k.
// Result layout differs: element e of lane (j + 16g) holds row g + 4e (f64) or
// row 4g + e (f32), column j (checked on gfx950 by an in-bounds probe).
template <> struct Mfma<double> {
  using V = dvec4;
  static __device__ __forceinline__ V mma(double a, double b, V c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int g, int e) { return g + 4 * e; }
};
template <> struct Mfma<float> {
  using V = fvec4;
  static __device__ __forceinline__ V mma(float a, float b, V c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int g, int e) { return 4 * g + e; }
};

constexpr int kT = 16;              // block size
constexpr int kLd = 17;             // padded LDS row stride (bank-conflict free column reads)
constexpr int kTL = kT * kLd;       // LDS words per tile
constexpr double kWFloor = 0.1;
constexpr double kReuseH = 1e-6;    // ||h||_inf below which a factor is reused

__device__ __forceinline__ int fold_x(int p, int nx) { return (p & 1) ? nx - 1 - (p >> 1) : (p >> 1); }
__device__ __forceinline__ int pos_of(int x, int nx) {
  return (2 * x <= nx - 1) ? 2 * x : 2 * (nx - 1 - x) + 1;
}
__device__ __forceinline__ int wrap(int x, int nx) { return x < 0 ? x + nx : (x >= nx ? x - nx : x); }

// value of lane `src` (wave-uniform) broadcast to every lane
__device__ __forceinline__ double lane_bcast(double v, int src) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), src);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), src);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float lane_bcast(float v, int src) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), src));
}

template <int BB, int NW, typename R>
struct BandShared {
  R P[BB + 1][kTL];        // panel blocks (S, then L after the panel solve)
  R PD[BB + 1][kTL];       // -S(J+d, J), the trailing update's right operand
  R NR[BB + 1][kTL];       // staging area of the entering block row
  R T[kTL];                // L_JJ^{-T} D_J^{-1}, then the diagonal block's inverse A_JJ^{-1}
  R X[kTL];                // L_JJ^{-1}
  double Dv[kT];
  double ring[(BB + 1) * kT];   // right-hand side / solution window of live block rows
  double newr[kT];
  double yJ[kT];
  double part[NW * kWave];
  double red[NW][4];
  int flag[4];
};

// Per-sample view: geometry, pointers, stencil coefficients.
struct Ctx {
  int nx, nt, m, n, M, NB;
  double q, c, cd;           // f-coefficient dt/(2dx), diffusion number, -1 + 2c
  bool god;                  // Godunov's interface flux (else Lax-Friedrichs)
  double sg, cv;             // Godunov form: dt/dx and nu dt/dx^2
  bool bwd;
  const double* uh;          // u_hat (forward)
  const double* g;           // upstream gradient (backward)
  double* u;                 // current iterate (forward) / u* (backward)
  double* lam;               // current multipliers (canonical order)
  unsigned char* ws;
};

// workspace layout of one sample (byte offsets, 256-aligned)
struct WsLayout {
  size_t hdr, L, Dg, Y, rin, rvec, lamp, p, t, res, z, acol, aval;
  size_t scol, sval, sepw, sepr;   // two-sided form: separator rows, exported updates
  size_t total;
};

// panels in flight in the forward and backward substitution sweeps
constexpr int kFwdDepth = 3, kBackDepth = 3;
constexpr int kContrib = 16;   // stencil contributions to one row of S (4 variables x 4 rows)

__host__ __device__ inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

__host__ __device__ inline int band_bb(int nx, int nt) {
  int b = nt > 2 ? nx + 2 : 4;
  if (b < 4) b = 4;
  return (b + kT - 1) / kT;
}

__host__ __device__ inline WsLayout ws_layout(int nx, int nt, int BB, size_t rsize) {
  WsLayout w;
  const size_t m = (size_t)nx * (nt - 1), n = (size_t)nx * nt;
  const size_t M = (m + kT - 1) / kT * kT, NB = M / kT;
  size_t o = 0;
  w.hdr = o; o += 256;
  w.L = o; o += align256(NB * (BB + 1) * 256 * rsize);
  w.Dg = o; o += align256(M * 8);
  w.Y = o; o += align256(M * 8);
  w.rin = o; o += align256(M * 8);
  w.rvec = o; o += align256(m * 8);
  w.lamp = o; o += align256(m * 8);
  w.p = o; o += align256(n * 8);
  w.t = o; o += align256(n * 8);
  w.res = o; o += align256(m * 8);
  w.z = o; o += align256(m * 8);        // second-order correction: S z = h(u + p)
  w.acol = o; o += align256(M * kContrib * 4);
  w.aval = o; o += align256(M * kContrib * 8);
  // two-sided form: the bottom sweep's copy of the separator rows' stencil
  // contributions, and each side's update of the separator (its lower block
  // triangle, BB(BB+1)/2 blocks, and its right-hand side)
  const size_t sr = (size_t)BB * kT, nsb = (size_t)BB * (BB + 1) / 2;
  w.scol = o; o += align256(sr * kContrib * 4);
  w.sval = o; o += align256(sr * kContrib * 8);
  w.sepw = o; o += align256(2 * nsb * 256 * 8);
  w.sepr = o; o += align256(2 * sr * 8);
  w.total = o;
  return w;
}

// ------------------------------------------------------------------ stencil
// d(v) = u - u_hat (forward), -g (backward)
__device__ __forceinline__ double dres(const Ctx& C, int v) {
  return C.bwd ? -C.g[v] : C.u[v] - C.uh[v];
}

__device__ __forceinline__ double jt_at(const Ctx& C, const double* y, int k, int x);

// residual entering the Schur right-hand side: the stationarity residual
// u - u_hat + J^T lam (forward; the system is solved for the multiplier
// increment, whose right-hand side vanishes at the solution), or -g (adjoint)
__device__ __forceinline__ double gres(const Ctx& C, int k, int x) {
  const int v = k * C.nx + x;
  return C.bwd ? -C.g[v] : C.u[v] - C.uh[v] + jt_at(C, C.lam, k, x);
}

// Godunov's flux of the convex f(u) = u^2/2 (paper Appendix D, Godunov's
// flux conservation) between a left state a and a right state b:
// F = max(f(max(a, 0)), f(min(b, 0))).  Newton steps differentiate the branch
// that attains the max (ties: the left state's), so F_a, F_b, F_aa, F_bb are
// the generalized derivatives of a semismooth Newton step; each branch is a
// square of one state, which keeps the Lagrangian Hessian diagonal.
struct GFlux {
  double F, Fa, Fb, Faa, Fbb;
};
__device__ __forceinline__ GFlux gflux(double a, double b) {
  const double ap = fmax(a, 0.0), bm = fmin(b, 0.0);
  GFlux g;
  if (ap * ap >= bm * bm) {
    g.F = 0.5 * ap * ap; g.Fa = ap; g.Fb = 0.0; g.Faa = a > 0.0 ? 1.0 : 0.0; g.Fbb = 0.0;
  } else {
    g.F = 0.5 * bm * bm; g.Fa = 0.0; g.Fb = bm; g.Faa = 0.0; g.Fbb = b < 0.0 ? 1.0 : 0.0;
  }
  return g;
}

// Godunov form: coefficients of row (k, x) on u(k, x-1), u(k, x), u(k, x+1)
// from slab k (U); fm / fp are the fluxes at x - 1/2 and x + 1/2
struct GRow {
  double cl, c0, cr;
};
__device__ __forceinline__ GRow grow_of(const Ctx& C, const GFlux& fm, const GFlux& fp) {
  return GRow{-C.sg * fm.Fa - C.cv, -1.0 + C.sg * (fp.Fa - fm.Fb) + 2.0 * C.cv, C.sg * fp.Fb - C.cv};
}
__device__ __forceinline__ GRow grow(const Ctx& C, const double* U, int x) {
  const double u0 = U[x];
  return grow_of(C, gflux(U[wrap(x - 1, C.nx)], u0), gflux(u0, U[wrap(x + 1, C.nx)]));
}
// coefficient of u(k, y) in row (k, y-1), row (k, y) and row (k, y+1)
__device__ __forceinline__ GRow gcol(const Ctx& C, const double* U, int y) {
  const double u0 = U[y];
  const GFlux fm = gflux(U[wrap(y - 1, C.nx)], u0), fp = gflux(u0, U[wrap(y + 1, C.nx)]);
  return GRow{C.sg * fm.Fb - C.cv, -1.0 + C.sg * (fp.Fa - fm.Fb) + 2.0 * C.cv, -C.sg * fp.Fa - C.cv};
}

// W at variable (k, x) from the current multipliers, before the floor
__device__ __forceinline__ double w_raw(const Ctx& C, int k, int x) {
  if (k > C.nt - 2) return 1.0;
  const double* L = C.lam + (size_t)k * C.nx;
  const int xm = wrap(x - 1, C.nx), xp = wrap(x + 1, C.nx);
  if (C.god) {
    const double* U = C.u + (size_t)k * C.nx;
    const double u0 = U[x];
    const GFlux fm = gflux(U[xm], u0), fp = gflux(u0, U[xp]);
    return 1.0 + C.sg * (fp.Faa * (L[x] - L[xp]) + fm.Fbb * (L[xm] - L[x]));
  }
  return 1.0 + C.q * (L[xm] - L[xp]);
}

__device__ __forceinline__ double w_at(const Ctx& C, int k, int x) { return fmax(w_raw(C, k, x), kWFloor); }

// h of row (k, x) given slab k's three values and u(k+1, x)
__device__ __forceinline__ double h_of(const Ctx& C, double um, double u0, double up, double un) {
  if (C.god)
    return un - u0 + C.sg * (gflux(u0, up).F - gflux(um, u0).F) - C.cv * (up - 2.0 * u0 + um);
  return un - u0 + 0.5 * C.q * (up * up - um * um) - C.c * (up - 2.0 * u0 + um);
}

// h of row (k, x)
__device__ __forceinline__ double h_row(const Ctx& C, int k, int x) {
  const double* U = C.u + (size_t)k * C.nx;
  return h_of(C, U[wrap(x - 1, C.nx)], U[x], U[wrap(x + 1, C.nx)], C.u[(size_t)(k + 1) * C.nx + x]);
}

// (J^T y)(k, x) for a row-space vector y in canonical order
__device__ __forceinline__ double jt_at(const Ctx& C, const double* y, int k, int x) {
  const int nx = C.nx;
  double s = 0.0;
  if (k >= 1) s += y[(size_t)(k - 1) * nx + x];
  if (k <= C.nt - 2) {
    const double* Y = y + (size_t)k * nx;
    if (C.god) {
      const GRow g = gcol(C, C.u + (size_t)k * nx, x);
      return s + g.cl * Y[wrap(x - 1, nx)] + g.c0 * Y[x] + g.cr * Y[wrap(x + 1, nx)];
    }
    const double uu = C.u[(size_t)k * nx + x];
    s += (C.q * uu - C.c) * Y[wrap(x - 1, nx)];     // row (k, x-1): its +1 neighbour is x
    s += C.cd * Y[x];
    s += (-C.q * uu - C.c) * Y[wrap(x + 1, nx)];    // row (k, x+1): its -1 neighbour is x
  }
  return s;
}

// (J z)(row k, x) for a variable-space vector z
__device__ __forceinline__ double j_at(const Ctx& C, const double* z, int k, int x) {
  const int nx = C.nx;
  const double* U = C.u + (size_t)k * nx;
  const double* Z = z + (size_t)k * nx;
  const int xp = wrap(x + 1, nx), xm = wrap(x - 1, nx);
  if (C.god) {
    const GRow g = grow(C, U, x);
    return z[(size_t)(k + 1) * nx + x] + g.c0 * Z[x] + g.cr * Z[xp] + g.cl * Z[xm];
  }
  return z[(size_t)(k + 1) * nx + x] + C.cd * Z[x] + (C.q * U[xp] - C.c) * Z[xp] +
         (-C.q * U[xm] - C.c) * Z[xm];
}

// ------------------------------------------------------------------ reductions
template <int NW>
__device__ __forceinline__ double block_sum(double v, double (*red)[4], int slot) {
  v = wave_sum(v);
  const int w = threadIdx.x / kWave;
  if ((threadIdx.x & (kWave - 1)) == 0) red[w][slot] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int q = 0; q < NW; ++q) s += red[q][slot];
  __syncthreads();
  return s;
}

template <int NW>
__device__ __forceinline__ double block_max(double v, double (*red)[4], int slot) {
  v = wave_max(v);
  const int w = threadIdx.x / kWave;
  if ((threadIdx.x & (kWave - 1)) == 0) red[w][slot] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int q = 0; q < NW; ++q) s = fmax(s, red[q][slot]);
  __syncthreads();
  return s;
}

// ------------------------------------------------------------------ assembly
// Row r (internal order) of S and of the right-hand side h - J W^{-1} d,
// scattered into the staging tile row `a` for columns [lo, hi) (block-aligned):
// S[r, r'] = sum over variables v of row r of J(r,v) J(r',v) / W(v).
// Contributions of row r (internal order) of S = J W^{-1} J^T and of the
// right-hand side h - J W^{-1} g: for each of the four variables v of row
// (k, x) and each row r' touching v, the value J(r,v) J(r',v) / W(v) with the
// column of r' (a column may appear more than once when Nx is tiny; the
// scatter adds them).  Computed for all rows in one parallel pass before the
// factorization, so the factorization only scatters prefetched pairs.
// Rows [r0, r1) go to entries r - base of (cols, vals); with `rhs` their
// right-hand sides are written too (rin and rvec).
template <int NW>
__device__ void assemble_rows(const Ctx& C, const WsLayout& WL, int r0, int r1, int* cols, double* vals,
                              int base, bool rhs_out) {
  double* rvec = (double*)(C.ws + WL.rvec);
  double* rin = (double*)(C.ws + WL.rin);
  const int nx = C.nx;
  for (int r = r0 + (int)threadIdx.x; r < r1; r += NW * kWave) {
    int* col = cols + (size_t)(r - base) * kContrib;
    double* val = vals + (size_t)(r - base) * kContrib;
    if (r >= C.m) {                    // padding row: identity
#pragma unroll
      for (int t = 0; t < kContrib; ++t) { col[t] = r; val[t] = t == 0 ? 1.0 : 0.0; }
      if (rhs_out) rin[r] = 0.0;
      continue;
    }
    const int k = r / nx, px = r - k * nx, x = fold_x(px, nx);
    double rhs = C.bwd ? 0.0 : h_row(C, k, x);
    const GRow gr = C.god ? grow(C, C.u + (size_t)k * nx, x) : GRow{0.0, 0.0, 0.0};
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      // the four variables of row (k, x): (k+1, x), (k, x), (k, x+1), (k, x-1)
      const int kk = (e == 0) ? k + 1 : k;
      const int y = (e <= 1) ? x : (e == 2 ? wrap(x + 1, nx) : wrap(x - 1, nx));
      const size_t v = (size_t)kk * nx + y;
      const double uy = C.u[v];
      const bool up = kk >= 1, own = kk <= C.nt - 2;
      double al, cm, c0, cp;    // J(r, v); J of rows (kk, y-1), (kk, y), (kk, y+1) at v
      if (C.god) {
        al = (e == 0) ? 1.0 : (e == 1 ? gr.c0 : (e == 2 ? gr.cr : gr.cl));
        const GRow gc = own ? gcol(C, C.u + (size_t)kk * nx, y) : GRow{0.0, 0.0, 0.0};
        cm = gc.cl; c0 = gc.c0; cp = gc.cr;
      } else {
        al = (e == 0) ? 1.0 : (e == 1 ? C.cd : (e == 2 ? C.q * uy - C.c : -C.q * uy - C.c));
        cm = C.q * uy - C.c; c0 = C.cd; cp = -C.q * uy - C.c;
      }
      const double sv = al / w_at(C, kk, y);
      rhs -= sv * gres(C, kk, y);
      // rows touching variable (kk, y): (kk-1, y) with 1; (kk, y-1), (kk, y), (kk, y+1)
      col[4 * e + 0] = up ? (kk - 1) * nx + pos_of(y, nx) : r;
      val[4 * e + 0] = up ? sv : 0.0;
      col[4 * e + 1] = own ? kk * nx + pos_of(wrap(y - 1, nx), nx) : r;
      val[4 * e + 1] = own ? sv * cm : 0.0;
      col[4 * e + 2] = own ? kk * nx + pos_of(y, nx) : r;
      val[4 * e + 2] = own ? sv * c0 : 0.0;
      col[4 * e + 3] = own ? kk * nx + pos_of(wrap(y + 1, nx), nx) : r;
      val[4 * e + 3] = own ? sv * cp : 0.0;
    }
    if (rhs_out) {
      rvec[(size_t)k * nx + x] = rhs;
      rin[r] = rhs;
    }
  }
  __syncthreads();
}

template <int NW>
__device__ void assemble_all(const Ctx& C, const WsLayout& WL) {
  assemble_rows<NW>(C, WL, 0, C.M, (int*)(C.ws + WL.acol), (double*)(C.ws + WL.aval), 0, true);
}

// Right-hand side h - J W^{-1} g alone (rvec canonical, rin internal order),
// for a Newton step solved with the factor of an earlier iteration.
template <int NW>
__device__ void assemble_rhs_rows(const Ctx& C, const WsLayout& WL, int r0, int r1) {
  double* rvec = (double*)(C.ws + WL.rvec);
  double* rin = (double*)(C.ws + WL.rin);
  const int nx = C.nx;
  for (int r = r0 + (int)threadIdx.x; r < r1; r += NW * kWave) {
    if (r >= C.m) { rin[r] = 0.0; continue; }
    const int k = r / nx, px = r - k * nx, x = fold_x(px, nx);
    double rhs = h_row(C, k, x);
    const GRow gr = C.god ? grow(C, C.u + (size_t)k * nx, x) : GRow{0.0, 0.0, 0.0};
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int kk = (e == 0) ? k + 1 : k;
      const int y = (e <= 1) ? x : (e == 2 ? wrap(x + 1, nx) : wrap(x - 1, nx));
      const double uy = C.u[(size_t)kk * nx + y];
      const double al = C.god ? ((e == 0) ? 1.0 : (e == 1 ? gr.c0 : (e == 2 ? gr.cr : gr.cl)))
                              : ((e == 0) ? 1.0 : (e == 1 ? C.cd : (e == 2 ? C.q * uy - C.c : -C.q * uy - C.c)));
      rhs -= al / w_at(C, kk, y) * gres(C, kk, y);
    }
    rvec[(size_t)k * nx + x] = rhs;
    rin[r] = rhs;
  }
  __syncthreads();
}

template <int NW>
__device__ void assemble_rhs(const Ctx& C, const WsLayout& WL) {
  assemble_rhs_rows<NW>(C, WL, 0, C.M);
}

// scatter the prefetched contributions of row a of block row I into the staging tile
template <int BB, typename R, int NC = kContrib>
__device__ __forceinline__ void scatter_row(int I, int a, const int* col, const double* val,
                                            R (*NR)[kTL]) {
  const int lo = (I - BB) * kT, hi = (I + 1) * kT;
#pragma unroll
  for (int t = 0; t < NC; ++t) {
    const int cc = col[t];
    if (cc >= lo && cc < hi) {
      const int cb = cc / kT;
      NR[I - cb][a * kLd + (cc - cb * kT)] += (R)val[t];
    }
  }
}

// The value itself, as a fresh scalar at this point of the program: offsets
// derived from it are recomputed here (one scalar add) instead of being hoisted
// out of the step loop, where four LDS addresses per accumulator slot would
// take the registers the accumulator window needs.
// (x must be uniform over the wavefront.)
__device__ __forceinline__ int fresh(int x) {
  x = __builtin_amdgcn_readfirstlane(x);
  asm volatile("" : "+s"(x));
  return x;
}

// the same for a per-lane value
__device__ __forceinline__ int fresh_v(int x) {
  asm volatile("" : "+v"(x));
  return x;
}

// ------------------------------------------------------------------ parts
// The two-sided form splits the block rows into a top part [0, K), a
// separator [K, K+BB) and a bottom part [K+BB, NB).  One workgroup factors the
// top downwards, another the bottom upwards (as the row-and-column reversed
// matrix, which has the same band).  The parts do not touch (their rows are
// more than BB blocks apart); each leaves its Schur complement update of the
// separator in the workspace, and a third sweep factors the separator (its
// own entries plus both updates) last.  That is the LDL^T factorization of S
// with the rows ordered top, bottom reversed, separator: the flops of the
// one-sided sweep, half its chain of dependent panel steps.
enum PartKind { kWhole = 0, kTop = 1, kBottom = 2, kSep = 3 };

struct Part {
  int kind;
  int K, Kb;     // first separator block row; block rows of the bottom part
  int steps;     // panel steps of the sweep
  int rows;      // block rows (sweep coordinates) that enter; later ones are zero
};

template <int BB>
__device__ __forceinline__ Part make_part(const Ctx& C, int kind) {
  Part P;
  P.kind = kind;
  P.K = (C.NB - BB) / 2;
  P.Kb = C.NB - P.K - BB;
  P.steps = kind == kWhole ? C.NB : (kind == kTop ? P.K : (kind == kBottom ? P.Kb : BB));
  P.rows = kind == kWhole ? C.NB : (kind == kTop ? P.K + BB : (kind == kBottom ? P.Kb + BB : BB));
  return P;
}

// block index under which panel J of a sweep stores L, D and y
__device__ __forceinline__ int part_slot(const Ctx& C, const Part& P, int J) {
  return P.kind == kBottom ? C.NB - 1 - J : (P.kind == kSep ? P.K + J : J);
}

constexpr int kNoCol = 0x3fffffff;   // a contribution the sweep leaves out

// Contributions t0 .. t0+NC-1 of row a of block row I, both in sweep
// coordinates.  The bottom sweep takes only a separator row's coupling to
// the bottom part; the rest of the separator rows is the top's.
template <int NC>
__device__ __forceinline__ void part_row(const Ctx& C, const WsLayout& WL, const Part& P, int I, int a, int t0,
                                         int* cl, double* vl) {
  if (I >= P.rows) {
#pragma unroll
    for (int t = 0; t < NC; ++t) { cl[t] = kNoCol; vl[t] = 0.0; }
    return;
  }
  if (P.kind != kBottom) {
    const size_t o = ((size_t)I * kT + a) * kContrib + t0;
    const int* col = (const int*)(C.ws + WL.acol) + o;
    const double* val = (const double*)(C.ws + WL.aval) + o;
#pragma unroll
    for (int t = 0; t < NC; ++t) { cl[t] = col[t]; vl[t] = val[t]; }
    return;
  }
  const int r = C.M - 1 - (I * kT + a);          // the row in the matrix's own order
  const bool sep = I >= P.Kb;
  const size_t o = (size_t)(sep ? r - P.K * kT : r) * kContrib + t0;
  const int* col = (const int*)(C.ws + (sep ? WL.scol : WL.acol)) + o;
  const double* val = (const double*)(C.ws + (sep ? WL.sval : WL.aval)) + o;
#pragma unroll
  for (int t = 0; t < NC; ++t) {
    const int c = C.M - 1 - col[t];
    cl[t] = (sep && c >= P.Kb * kT) ? kNoCol : c;
    vl[t] = val[t];
  }
}

// right-hand side of row a of block row I (sweep coordinates)
__device__ __forceinline__ long part_rhs_index(const Ctx& C, const Part& P, int I, int a) {
  if (I >= P.rows) return -1;
  if (P.kind == kBottom) return I < P.Kb ? C.M - 1 - (I * kT + a) : -1;
  return (long)I * kT + a;
}

__device__ __forceinline__ double part_rhs(const Ctx& C, const double* rin, const Part& P, int I, int a) {
  const long i = part_rhs_index(C, P, I, a);
  return i < 0 ? 0.0 : rin[i];
}

// Entry [a][b] of separator block (i, i - d) (local block rows): the top's
// export holds the separator's entries with the top's update, the bottom's
// its own update in reversed coordinates, where the block is
// (BB-1-(i-d), same d) and the entry [15-b][15-a].
template <int BB>
__device__ __forceinline__ double sep_entry(const double* sw, int i, int d, int a, int b) {
  constexpr int NSB = BB * (BB + 1) / 2;
  const int ib = BB - 1 - (i - d);
  return sw[(size_t)(i * (i + 1) / 2 + d) * 256 + a * kT + b] +
         sw[(size_t)(NSB + ib * (ib + 1) / 2 + d) * 256 + (15 - b) * kT + (15 - a)];
}

// separator right-hand side, local row i, entry a (both sides' exports)
template <int BB>
__device__ __forceinline__ double sep_rhs(const double* sr, int i, int a) {
  return sr[i * kT + a] + sr[BB * kT + (BB - 1 - i) * kT + (15 - a)];
}

// ------------------------------------------------------------------ factor
// Factor S (or the part PT of its two-sided form; the rows are assembled by
// the caller) with the fused forward substitution of the right-hand side;
// writes L blocks, D and y = L^{-1} r, and a top or bottom part exports its
// update of the separator.  Returns 1 if a non-positive pivot was met.
template <int BB, int NW, typename R>
__device__ __attribute__((always_inline)) int factor_sweep(const Ctx& C, const WsLayout& WL, BandShared<BB, NW, R>& sh,
                                                          const Part& PT) {
  using V = typename Mfma<R>::V;
  constexpr int NS = (BB + 1) * (BB + 2) / 2;
  constexpr int SPW = (NS + NW - 1) / NW;
  const int lane = threadIdx.x & (kWave - 1);
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);   // wave-uniform
  const int li = lane & 15, lk = lane >> 4;
  R* Lg = (R*)(C.ws + WL.L);
  double* Dg = (double*)(C.ws + WL.Dg);
  double* Y = (double*)(C.ws + WL.Y);
  double* rvec = (double*)(C.ws + WL.rvec);
  double* rin = (double*)(C.ws + WL.rin);

  // slot metadata: slot id = w + NW*s -> (d, sidx)
  int sd[SPW], ss[SPW];
#pragma unroll
  for (int s = 0; s < SPW; ++s) {
    int id = w + NW * s;
    int d = -1, sidx = 0;
    if (id < NS) {
      int base = 0;
      for (int dd = 0; dd <= BB; ++dd) {
        int cnt = BB + 1 - dd;
        if (id < base + cnt) { d = dd; sidx = id - base; break; }
        base += cnt;
      }
    }
    sd[s] = d; ss[s] = sidx;
  }
  auto slot_row = [&](int s, int J) -> int {   // block row I held by slot s at step J
    const int d = sd[s], P = BB + 1 - d;
    int t = (ss[s] - J - d) % P;
    if (t < 0) t += P;
    return J + d + t;
  };
  // tr[s] = (I - J - d) for the block held by slot s at the current step J:
  // 0 means the slot holds a panel block; it decreases by one per step
  // (cyclically, period BB+1-d), so no division is needed inside the loop
  int tr[SPW];
#pragma unroll
  for (int s = 0; s < SPW; ++s) tr[s] = sd[s] >= 0 ? slot_row(s, 0) - sd[s] : 0;
  auto advance = [&]() {
#pragma unroll
    for (int s = 0; s < SPW; ++s) tr[s] = tr[s] == 0 ? BB - sd[s] : tr[s] - 1;
  };

  V acc[SPW];
#pragma unroll
  for (int s = 0; s < SPW; ++s) acc[s] = V{0, 0, 0, 0};

  auto zero_nr = [&]() {
    R* z = &sh.NR[0][0];
    for (int i = threadIdx.x; i < (BB + 1) * kTL; i += NW * kWave) z[i] = (R)0;
  };
  auto load_nr = [&](int s, int d) {
    V v;
#pragma unroll
    for (int e = 0; e < 4; ++e) v[e] = sh.NR[d][Mfma<R>::row(lk, e) * kLd + li];
    acc[s] = v;
  };

  const double* sw_in = (const double*)(C.ws + WL.sepw);
  const double* sr_in = (const double*)(C.ws + WL.sepr);
  // wavefront 1, lanes 0..15: row `lane` of the entering block row I, loaded
  // while wavefront 0 factors the diagonal block (which hides the latency)
  auto enter_row = [&](int I) {
    if (I < PT.rows) {
      // two halves of eight contributions bound the registers this needs
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        int cl[kContrib / 2];
        double vl[kContrib / 2];
        part_row<kContrib / 2>(C, WL, PT, I, lane, h * (kContrib / 2), cl, vl);
        scatter_row<BB, R, kContrib / 2>(I, lane, cl, vl, sh.NR);
      }
      sh.newr[lane] = part_rhs(C, rin, PT, I, lane);
    } else {
      sh.newr[lane] = 0.0;
    }
  };
  (void)rvec;

  // ---- initial window: block rows 0..BB
  for (int I = 0; I <= BB; ++I) {
    zero_nr();
    lds_barrier();
    if (PT.kind == kSep) {
      // the separator's block row I: both sides' exports (blocks left of the
      // separator were eliminated by the sides)
      if (I < BB) {
        for (int e = threadIdx.x; e < (I + 1) * 256; e += NW * kWave) {
          const int d = e >> 8, a = (e >> 4) & 15, b = e & 15;
          sh.NR[d][a * kLd + b] = (R)sep_entry<BB>(sw_in, I, d, a, b);
        }
      }
      if (threadIdx.x < kT)
        sh.ring[(I % (BB + 1)) * kT + threadIdx.x] = I < BB ? sep_rhs<BB>(sr_in, I, threadIdx.x) : 0.0;
    } else if (threadIdx.x < kT) {
      int cl[kContrib];
      double vl[kContrib];
      part_row<kContrib>(C, WL, PT, I, threadIdx.x, 0, cl, vl);
      scatter_row<BB, R>(I, threadIdx.x, cl, vl, sh.NR);
      sh.ring[(I % (BB + 1)) * kT + threadIdx.x] = part_rhs(C, rin, PT, I, threadIdx.x);
    }
    lds_barrier();
#pragma unroll
    for (int s = 0; s < SPW; ++s)
      if (sd[s] >= 0 && sd[s] <= I && slot_row(s, 0) == I) load_nr(s, sd[s]);
    lds_barrier();
  }

  int bad = 0;
  for (int J = 0; J < PT.steps; ++J) {
    const int sl = part_slot(C, PT, J);
    // (a) gather the panel column J into LDS; clear the staging area
#pragma unroll
    for (int s = 0; s < SPW; ++s) {
      if (sd[s] < 0) continue;
      if (tr[s] == 0) {
        const int d = fresh(sd[s]);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          sh.P[d][Mfma<R>::row(lk, e) * kLd + li] = acc[s][e];
          if (d > 0) sh.PD[d][Mfma<R>::row(lk, e) * kLd + li] = -acc[s][e];
        }
      }
    }
    zero_nr();
    lds_barrier();

    // (b) wavefront 0: LDL^T of the diagonal block; wavefront 1: next block row
    if (w == 0) {
      // LDL^T of the symmetric 16x16 diagonal block A in registers.  Lanes
      // 0..15 hold column k = lane of the working matrix (v[i] = A[i][k]);
      // lanes 16..31 hold column k = lane - 16 of the identity.  Pivot p
      // broadcasts column p from lane p and every lane applies the same row
      // operation v[i] -= (A[i][p] / D_p) v[p], so the matrix lanes eliminate
      // while the identity lanes turn into the columns of X = L^{-1}.  Row p
      // of X is final after pivot p: X and T = L^{-T} D^{-1} go to LDS as the
      // sweep goes, and the wavefront then forms A^{-1} = T X on MFMA.  The
      // stored factor holds A^{-1} and M(J+d) = L(J+d, J) L^{-1} = S(J+d, J)
      // A^{-1}: the substitutions then run on z = L y (the right-hand side
      // minus the earlier panels' updates, no diagonal solve in the chain),
      // z(J+d) -= M(J+d) z(J) forward and x(J) = A^{-1} z(J) - sum M^T x
      // backward.  (Lanes 32..63 repeat lanes 0..31.)
      const int k = fresh_v(lane & (kT - 1));  // (not hoisted: 16 identity values would be)
      const bool xl = (lane & 16) != 0;        // an identity / X lane
      // The elimination runs in the factor's precision R: an FP32 factor
      // (refined in FP64 by its solves) takes FP32 pivots, one readlane per
      // broadcast value instead of two.
      double dmine = 1.0;
      int nonpos = 0;
      R v[kT];
#pragma unroll
      for (int i = 0; i < kT; ++i) v[i] = xl ? (i == k ? (R)1 : (R)0) : sh.P[0][i * kLd + k];
      const double zk = sh.ring[(J % (BB + 1)) * kT + k];   // z(J), final
      R* Lgd = Lg + ((size_t)sl * (BB + 1)) * 256;
#pragma unroll
      for (int p = 0; p < kT; ++p) {
        const R dp = lane_bcast(v[p], p);        // A[p][p]
        nonpos |= !(dp > (R)0);
        const R rdp = rcp_nr(dp);
        if (k == p) dmine = dp;
        const R m = v[p] * rdp;                  // A lanes: L[k][p] = A[p][k] / D_p (symmetry)
#pragma unroll
        for (int i = p + 1; i < kT; ++i) v[i] -= lane_bcast(v[i], p) * m;
        if (xl && lane < 32) {                   // row p of X is final
          sh.T[k * kLd + p] = v[p] * rdp;        // T[k][p] = X[p][k] / D_p
          sh.X[p * kLd + k] = v[p];
        }
      }
      if (lane < kT) {
        sh.Dv[k] = dmine;
        Dg[(size_t)sl * kT + k] = dmine;
        sh.yJ[k] = zk;
        Y[(size_t)sl * kT + k] = zk;
      }
      if (lane == 0 && nonpos) sh.flag[0] = 1;
      // A^{-1} = T X (one wavefront; T is overwritten only after every lane
      // has read its operands, which the product's result depends on)
      V ai = V{0, 0, 0, 0};
#pragma unroll
      for (int qq = 0; qq < 4; ++qq)
        ai = Mfma<R>::mma(sh.T[li * kLd + 4 * qq + lk], sh.X[(4 * qq + lk) * kLd + li], ai);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        sh.T[Mfma<R>::row(lk, e) * kLd + li] = ai[e];
        Lgd[Mfma<R>::row(lk, e) * kT + li] = ai[e];
      }
    } else if (w == 1 && lane < kT) {
      enter_row(J + BB + 1);           // entering block row J+BB+1
    }
    lds_barrier();

    // (c) panel solve M(J+d) = S(J+d, J) A^{-1} for d >= 1
#pragma unroll
    for (int s = 0; s < SPW; ++s) {
      if (sd[s] < 1) continue;
      if (tr[s] != 0) continue;
      const int d = fresh(sd[s]);
      V res = V{0, 0, 0, 0};
#pragma unroll
      for (int qq = 0; qq < 4; ++qq) {
        const R av = sh.P[d][li * kLd + 4 * qq + lk];
        const R bv = sh.T[(4 * qq + lk) * kLd + li];
        res = Mfma<R>::mma(av, bv, res);
      }
      R* Lgd = Lg + ((size_t)sl * (BB + 1) + d) * 256;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        sh.P[d][Mfma<R>::row(lk, e) * kLd + li] = res[e];
        Lgd[Mfma<R>::row(lk, e) * kT + li] = res[e];
      }
    }
    lds_barrier();

    // (d) forward-substitution update, trailing update, entering row
    for (int t = threadIdx.x; t < kT * BB; t += NW * kWave) {
      const int d = 1 + t / kT, a = t - (d - 1) * kT;
      const int I = J + d;
      if (I < PT.rows) {
        double s = 0.0;
#pragma unroll
        for (int cc = 0; cc < kT; ++cc) s += (double)sh.P[d][a * kLd + cc] * sh.yJ[cc];
        sh.ring[(I % (BB + 1)) * kT + a] -= s;
      }
    }
#pragma unroll
    for (int s = 0; s < SPW; ++s) {
      if (sd[s] < 0) continue;
      if (tr[s] == 0) {
        load_nr(s, fresh(sd[s]));            // retire panel block, take the entering one
      } else {
        const int dk = tr[s], di = tr[s] + fresh(sd[s]);  // K - J and I - J: 1 <= dk <= di <= BB
        V v = acc[s];
#pragma unroll
        for (int qq = 0; qq < 4; ++qq) {
          const R av = sh.P[di][li * kLd + 4 * qq + lk];
          const R bv = sh.PD[dk][li * kLd + 4 * qq + lk];
          v = Mfma<R>::mma(av, bv, v);
        }
        acc[s] = v;
      }
      // keep the scheduler from hoisting every slot's operand loads at once
      __builtin_amdgcn_sched_barrier(0);
    }
    if (threadIdx.x < kT) sh.ring[(J % (BB + 1)) * kT + threadIdx.x] = sh.newr[threadIdx.x];
    advance();
    lds_barrier();
  }
  if (PT.kind == kTop || PT.kind == kBottom) {
    // export the window's separator blocks (local row d + tr, diagonal d) and
    // the separator's right-hand side
    constexpr int NSB = BB * (BB + 1) / 2;
    double* sw = (double*)(C.ws + WL.sepw) + (PT.kind == kBottom ? (size_t)NSB * 256 : 0);
    double* sr = (double*)(C.ws + WL.sepr) + (PT.kind == kBottom ? BB * kT : 0);
#pragma unroll
    for (int s = 0; s < SPW; ++s) {
      if (sd[s] < 0) continue;
      const int d = fresh(sd[s]), il = d + tr[s];
      if (il >= BB) continue;
      double* blk = sw + (size_t)(il * (il + 1) / 2 + d) * 256;
#pragma unroll
      for (int e = 0; e < 4; ++e) blk[Mfma<R>::row(lk, e) * kT + li] = (double)acc[s][e];
    }
    for (int i = threadIdx.x; i < BB * kT; i += NW * kWave)
      sr[i] = sh.ring[((PT.steps + i / kT) % (BB + 1)) * kT + (i % kT)];
  }
  bad = sh.flag[0];
  __syncthreads();            // factor (global) visible to the sweeps
  if (threadIdx.x == 0) sh.flag[0] = 0;
  lds_barrier();
  return bad;
}

// ------------------------------------------------------------------ solves
// The stored factor of panel J holds A_JJ^{-1} (block 0) and M(J+d) =
// L(J+d, J) L_JJ^{-1} (blocks d = 1..BB); Y holds z = L y.
//
// Forward substitution z(J+d) -= M(J+d) z(J) on the right-hand side rin (the
// whole matrix, or the part PT of its two-sided form: a top or bottom part
// exports its update of the separator's right-hand side, the separator's
// sweep starts from both).  Thread t < 16*BB owns row t % 16 of M(J+1+t/16)
// and updates that row of the window; the thread of d = BB starts its row
// (block row J+BB enters) from the right-hand side.  One barrier per panel
// step: step J reads only z(J), which the previous step's barrier made final,
// and writes the rows J+1..J+BB.
//
// Both sweeps keep the loads of the next few panels (kFwdDepth, kBackDepth)
// in flight: a stage is refilled right after its step, every load is in
// bounds and unconditional (values a step does not need are masked where they
// are used), so each step waits only for the stage it consumes and the HBM
// latency overlaps the dependent chain of the steps in between.
template <int BB, int NW, typename R>
__device__ __attribute__((always_inline)) void forward_sweep(
    const Ctx& C, const WsLayout& WL, BandShared<BB, NW, R>& sh, const double* rin, double* Y, const Part& PT) {
  static_assert(NW * kWave >= kT * BB, "forward sweep needs 16*BB threads");
  const R* Lg = (const R*)(C.ws + WL.L);
  // (fresh: the thread-derived offsets below are formed inside each sweep,
  // not hoisted into registers held across a caller's refinement loop)
  const int t = fresh_v(threadIdx.x);
  const bool offd = t < kT * BB;
  // threads past 16*BB load (and never use) a row of block 1
  const int d = offd ? 1 + t / kT : 1, a = t % kT;
  const double* sr_in = (const double*)(C.ws + WL.sepr);
  for (int i = t; i < (BB + 1) * kT; i += NW * kWave) {
    const int I = i / kT, aa = i - I * kT;
    // rows 0..BB-1; row BB enters at step 0
    sh.ring[i] = I >= BB ? 0.0
                         : (PT.kind == kSep ? sep_rhs<BB>(sr_in, I, aa) : part_rhs(C, rin, PT, I, aa));
  }
  // one pipeline stage: this thread's row of M(J+d) and the right-hand side
  // entry of block row J+BB (the row that enters at step J)
  struct Stage {
    R l[kT];
    double r;
  };
  Stage st[kFwdDepth];
  const int last = PT.steps - 1;
  auto load = [&](int J, Stage& s) {
    const int Jc = J < last ? J : last;        // stages past the last panel are never used
    const R* src = Lg + ((size_t)part_slot(C, PT, Jc) * (BB + 1) + d) * 256 + a * kT;
#pragma unroll
    for (int c = 0; c < kT; ++c) s.l[c] = src[c];
    const long ri = part_rhs_index(C, PT, Jc + BB, a);
    s.r = rin[ri < 0 ? 0 : ri];
  };
  auto step = [&](int J, const Stage& s) {
    const double* zJ = &sh.ring[(J % (BB + 1)) * kT];
    if (t < kT) Y[(size_t)part_slot(C, PT, J) * kT + t] = zJ[t];
    if (offd && J + d < PT.rows) {
      double sum = 0.0;
#pragma unroll
      for (int c = 0; c < kT; ++c) sum += (double)s.l[c] * zJ[c];
      double* zr = &sh.ring[((J + d) % (BB + 1)) * kT + a];
      if (d == BB)
        *zr = (part_rhs_index(C, PT, J + BB, a) >= 0 ? s.r : 0.0) - sum;   // (the slot of row J-1)
      else
        *zr -= sum;
    }
    lds_barrier();
  };
  if (PT.steps > 0) {
    // stages filled in the order the loop refills them, so the wait before
    // each step covers that stage's loads only
#pragma unroll
    for (int b = 0; b < kFwdDepth; ++b) {
      load(b, st[b]);
      __builtin_amdgcn_sched_barrier(0);
    }
    lds_barrier();
    // whole rounds of kFwdDepth steps (one loop exit, which keeps the
    // compiler's wait before each step to that step's stage); steps past the
    // last panel are skipped
    for (int J0 = 0; J0 < PT.steps; J0 += kFwdDepth) {
#pragma unroll
      for (int b = 0; b < kFwdDepth; ++b) {
        const int J = J0 + b;
        if (J < PT.steps) step(J, st[b]);
        load(J + kFwdDepth, st[b]);
      }
    }
  }
  lds_barrier();
  if (PT.kind == kTop || PT.kind == kBottom) {
    double* sr = (double*)(C.ws + WL.sepr) + (PT.kind == kBottom ? BB * kT : 0);
    for (int i = t; i < BB * kT; i += NW * kWave) sr[i] = sh.ring[((PT.steps + i / kT) % (BB + 1)) * kT + (i % kT)];
  }
  __syncthreads();            // Y visible to every wavefront
}

// backward substitution x(J) = A_JJ^{-1} z(J) - sum_d M(J+d)^T x(J+d); x is
// written in canonical row order.  Thread (c = t % 16, g = t / 16) accumulates
// the (d, a) pairs pq = g, g + NG, ... (d = pq / 16, a = pq % 16) of
// sum_a A^{-1}[a][c] z[a] - sum_{d >= 1, a} M(J+d)[a][c] x(J+d)[a], taking
// z[a] of its d = 0 pair from the stage; lanes 0..15 add the NG partial sums.
// Panels jhi down to jlo; blocks at rows >= nbr are absent.  rev: the bottom
// part's reversed coordinates (panel J stored as block NB-1-J).  keep_ring:
// the window already holds x of rows jhi+1 .. jhi+BB.  Rows are written to
// xout (canonical order, plus addlam when given) only with write_x.
struct BackRange {
  int jhi, jlo, nbr;
  bool rev, keep_ring, write_x;
  const double* addlam;
};

template <int BB, int NW, typename R>
__device__ __attribute__((always_inline)) void backward_sweep(
    const Ctx& C, const WsLayout& WL, BandShared<BB, NW, R>& sh, const double* Y, double* xout,
    const BackRange& BR) {
  constexpr int NT = NW * kWave;
  constexpr int NG = NT / kT;                            // 16-thread groups
  constexpr int NP = (BB + 1) * kT;                      // (d, a) pairs
  constexpr int NPQ = (NP + NG - 1) / NG;                // pairs per thread
  static_assert(NG >= kT, "the d = 0 pairs are every thread's first");
  const R* Lg = (const R*)(C.ws + WL.L);
  // (fresh: the thread-derived offsets below are formed inside each sweep,
  // not hoisted into registers held across a caller's refinement loop)
  const int t = fresh_v(threadIdx.x);
  const int cc = t & 15, grp = t >> 4;
  if (!BR.keep_ring)
    for (int i = t; i < (BB + 1) * kT; i += NT) sh.ring[i] = 0.0;
  // element offsets of the thread's (d, a) pairs inside a panel's blocks; a
  // spare pair (past the last) reads an entry it does not use
  unsigned off[NPQ];
#pragma unroll
  for (int i = 0; i < NPQ; ++i) {
    const int pq = grp + NG * i < NP ? grp + NG * i : NP - 1;
    off[i] = (unsigned)((pq / kT) * 256 + (pq % kT) * kT + cc);
  }
  // one pipeline stage: the thread's entries of panel J, z[g % 16] of its
  // d = 0 pair, and for row J*16 + (t % 16) the canonical index (-1 past the
  // last row) and the multiplier to add, read before the row is written
  // (addlam may be xout itself)
  struct Stage {
    R l[NPQ];
    double zz, al;
    int ci;
  };
  Stage st[kBackDepth];
  const double* alsrc = BR.addlam ? BR.addlam : Y;  // any valid address when there is none
  auto load = [&](int J, Stage& s) {
    const int Jc = J < BR.jlo ? BR.jlo : J;        // stages past the last panel are never used
    const unsigned sl = BR.rev ? C.NB - 1 - Jc : Jc;
    const R* base = Lg + (size_t)sl * (BB + 1) * 256;
#pragma unroll
    for (int i = 0; i < NPQ; ++i) s.l[i] = base[off[i]];
    s.zz = Y[sl * kT + (grp & 15)];
    const int r = BR.rev ? C.M - 1 - (Jc * kT + cc) : Jc * kT + cc;
    int ci = -1;
    if (r < C.m) {
      const int k = r / C.nx, px = r - k * C.nx;
      ci = k * C.nx + fold_x(px, C.nx);
    }
    s.ci = ci;
    s.al = alsrc[ci < 0 ? 0 : ci];
  };
  auto step = [&](int J, const Stage& s) {
    const int jm = J % (BB + 1);
    double sum = 0.0;
#pragma unroll
    for (int i = 0; i < NPQ; ++i) {
      // only the first pair can have d = 0 (pq >= NG >= 16 after it).  Rows
      // at or past nbr need no mask: their window entries are zero (never
      // written) and their stored blocks are zero.  A spare pair's entry is
      // masked in the register, so every window read is unconditional.
      const int pq = grp + NG * i;
      const int d = pq / kT, a = pq % kT;
      const int dd = d <= BB ? d : BB;
      const int slot = jm + dd > BB ? jm + dd - (BB + 1) : jm + dd;
      const double xv = sh.ring[slot * kT + a];
      const double lv = pq < NP ? (double)s.l[i] : 0.0;
      sum += lv * (i == 0 && d == 0 ? s.zz : -xv);
    }
    sh.part[t] = sum;
    lds_barrier();
    if (t < kT) {
      double x = 0.0;
      for (int q = 0; q < NG; ++q) x += sh.part[q * kT + t];
      sh.ring[jm * kT + t] = x;
      if (BR.write_x && s.ci >= 0) xout[s.ci] = BR.addlam ? x + s.al : x;
    }
    lds_barrier();
  };
  if (BR.jhi >= BR.jlo) {
    // stages filled in the order the loop refills them (as in the forward sweep)
#pragma unroll
    for (int b = 0; b < kBackDepth; ++b) {
      load(BR.jhi - b, st[b]);
      __builtin_amdgcn_sched_barrier(0);
    }
    lds_barrier();
    // whole rounds of kBackDepth steps (one loop exit, as in the forward sweep)
    for (int J0 = BR.jhi; J0 >= BR.jlo; J0 -= kBackDepth) {
#pragma unroll
      for (int b = 0; b < kBackDepth; ++b) {
        const int J = J0 - b;
        if (J >= BR.jlo) step(J, st[b]);
        load(J - kBackDepth, st[b]);
      }
    }
  }
  __syncthreads();            // x visible to every wavefront
}

// res = rvec - S x (float64, matrix free), x canonical; returns max |res|
template <int NW>
__device__ double schur_residual(const Ctx& C, const WsLayout& WL, const double* x, double* res,
                                 double (*red)[4]) {
  double* tv = (double*)(C.ws + WL.t);
  const double* rvec = (const double*)(C.ws + WL.rvec);
  for (int v = threadIdx.x; v < C.n; v += NW * kWave) {
    const int k = v / C.nx, xx = v - k * C.nx;
    tv[v] = jt_at(C, x, k, xx) / w_at(C, k, xx);
  }
  __syncthreads();
  double mx = 0.0;
  for (int r = threadIdx.x; r < C.m; r += NW * kWave) {
    const int k = r / C.nx, xx = r - k * C.nx;
    const double v = rvec[r] - j_at(C, tv, k, xx);
    res[r] = v;
    mx = fmax(mx, fabs(v));
  }
  return block_max<NW>(mx, red, 0);
}

// canonical row vector -> internal-order right-hand side
template <int NW>
__device__ void to_internal(const Ctx& C, const double* canon, double* rin) {
  for (int r = threadIdx.x; r < C.M; r += NW * kWave) {
    double v = 0.0;
    if (r < C.m) {
      const int k = r / C.nx, px = r - k * C.nx;
      v = canon[(size_t)k * C.nx + fold_x(px, C.nx)];
    }
    rin[r] = v;
  }
  __syncthreads();
}

// Solve S x = rhs given the factor (rhs in rin / rvec; y of the fused forward
// pass already in Y when have_y), with float64 iterative refinement in the
// mixed form.  Each sweep has a single call site.
template <int BB, int NW, typename R>
__device__ __attribute__((always_inline)) int solve_with_factor(
    const Ctx& C, const WsLayout& WL, BandShared<BB, NW, R>& sh, bool have_y, double* x,
    int max_refine = 6, double abs_floor = 0.0, bool stale = false) {
  double* Y = (double*)(C.ws + WL.Y);
  double* rin = (double*)(C.ws + WL.rin);
  double* res = (double*)(C.ws + WL.res);
  double* dx = (double*)(C.ws + WL.t);          // correction (t is free between residuals)
  const double* rvec = (const double*)(C.ws + WL.rvec);
  // the plain form refines only with a factor of an earlier iterate (stale)
  const bool plain = sizeof(R) == sizeof(double) && !stale;
  const Part whole = make_part<BB>(C, kWhole);
  const BackRange back{C.NB - 1, 0, C.NB, false, false, true, nullptr};
  double rn = 0.0;
  if (!plain) {
    for (int r = threadIdx.x; r < C.m; r += NW * kWave) rn = fmax(rn, fabs(rvec[r]));
    rn = block_max<NW>(rn, sh.red, 1);
  }
  int refines = 0;
  for (int it = 0; it <= max_refine; ++it) {
    if (it > 0 || !have_y) forward_sweep<BB, NW, R>(C, WL, sh, rin, Y, whole);
    backward_sweep<BB, NW, R>(C, WL, sh, Y, it == 0 ? x : dx, back);
    if (it > 0) {
      for (int r = threadIdx.x; r < C.m; r += NW * kWave) x[r] += dx[r];
      __syncthreads();
      ++refines;
    }
    if (plain || it == max_refine) break;
    const double rm = schur_residual<NW>(C, WL, x, res, sh.red);
    if (!(rm > fmax(1e-13 * rn, abs_floor))) break;
    to_internal<NW>(C, res, rin);
  }
  return refines;
}

// ------------------------------------------------------------------ kernels
// The Newton loop is a fixed sequence of launches (init, then max_newton rounds
// of factor / solve / step / eval, then finish), each kernel one workgroup per
// sample.  Per-sample progress lives in the workspace header, so samples that
// have converged (or failed) return at once from every later launch; the call
// never synchronizes with the host.  Splitting the loop keeps each kernel's
// live state small (the factorization's accumulator window needs most of the
// register file).

// per-sample state at the start of the sample's workspace block
struct BandState {
  int phase;        // 0 iterating, 1 converged and waiting for the final factor, 2 finished
  int status;       // SNAP_ST_*
  int iters, backtracks, refines;
  int factor_ok;    // 1 when the stored factor was taken at the returned point
  int factored;     // a factor of S from an earlier iteration is in the workspace
  int reuse;        // this iteration's step is solved with that factor
  int side_bad[2];  // two-sided form: a side's sweep met a non-positive pivot
  int adj_bad;      // two-sided adjoint: its factorization met one
  int round;        // two-sided form: a parallel refinement round of the step is due
  int soc_try;      // the full step failed and raised ||h||_1: band_soc tries a correction
  double soc_dd, soc_pp;   // (u - u_hat).p and p.p of that step
  double mu, uscale, h1, hinf, stinf;
};
static_assert(sizeof(BandState) <= 256, "state must fit the header");

__device__ __forceinline__ Ctx make_ctx(const KernelArgs& A, const snap_sample_desc& D, int sid, bool bwd) {
  Ctx C;
  C.nx = D.nx; C.nt = D.nt;
  C.m = D.nx * (D.nt - 1);
  C.n = D.nx * D.nt;
  C.M = (C.m + kT - 1) / kT * kT;
  C.NB = C.M / kT;
  C.q = 0.5 * D.dt / D.dx;
  C.c = D.p1 * D.dt / (2.0 * D.dx) + D.p0 * D.dt / (D.dx * D.dx);
  C.cd = -1.0 + 2.0 * C.c;
  C.god = D.family == SNAP_BURGERS_GODUNOV;
  C.sg = D.dt / D.dx;
  C.cv = D.p0 * D.dt / (D.dx * D.dx);
  C.bwd = bwd;
  C.uh = A.uhat ? A.uhat + D.var_off : nullptr;
  C.g = A.grad_u ? A.grad_u + D.var_off : nullptr;
  C.u = A.u + D.var_off;
  C.lam = A.lam + D.row_off;
  C.ws = A.ws + A.ws_off[sid];
  return C;
}

#define SNAP_BAND_KERNEL __global__ __launch_bounds__(NW * kWave) __attribute__((amdgpu_waves_per_eu(2, 2)))

// u = u_hat, lam = 0, state reset
template <int BB, int NW, typename R>
SNAP_BAND_KERNEL void band_init(KernelArgs A) {
  const int sid = A.order[blockIdx.x];
  const snap_sample_desc D = A.descs[sid];
  __shared__ double red[NW][4];
  const Ctx C = make_ctx(A, D, sid, false);
  const WsLayout WL = ws_layout(C.nx, C.nt, BB, sizeof(R));
  BandState* S = (BandState*)(C.ws + WL.hdr);
  double umax = 0.0;
  int nonfin = 0;
  for (int v = threadIdx.x; v < C.n; v += NW * kWave) {
    const double x = C.uh[v];
    C.u[v] = x;
    umax = fmax(umax, fabs(x));
    nonfin |= !finite(x);
  }
  for (int r = threadIdx.x; r < C.m; r += NW * kWave) C.lam[r] = 0.0;
  const double um = block_max<NW>(umax, red, 0);
  const double nf = block_max<NW>((double)nonfin, red, 1);
  if (threadIdx.x == 0) {
    BandState st{};
    st.phase = nf > 0.0 ? 2 : 0;
    st.status = nf > 0.0 ? SNAP_ST_NONFINITE : SNAP_ST_MAX_ITER;
    st.uscale = 1.0 + um;
    *S = st;
  }
}

// h, stationarity, convergence test at (u, lam)
template <int BB, int NW, typename R>
SNAP_BAND_KERNEL void band_eval(KernelArgs A) {
  const int sid = A.order[blockIdx.x];
  const snap_sample_desc D = A.descs[sid];
  __shared__ double red[NW][4];
  const Ctx C = make_ctx(A, D, sid, false);
  const WsLayout WL = ws_layout(C.nx, C.nt, BB, sizeof(R));
  BandState* S = (BandState*)(C.ws + WL.hdr);
  if (S->phase != 0) return;
  const bool keep = (A.opt.flags & SNAP_FLAG_KEEP_FACTOR) != 0;
  double hm = 0.0, h1 = 0.0, sm = 0.0;
  for (int v = threadIdx.x; v < C.n; v += NW * kWave) {
    const int k = v / C.nx, x = v - k * C.nx;
    sm = fmax(sm, fabs(dres(C, v) + jt_at(C, C.lam, k, x)));
    if (k <= C.nt - 2) {
      const double h = h_row(C, k, x);
      hm = fmax(hm, fabs(h));
      h1 += fabs(h);
      if (!finite(h)) hm = __builtin_nan("");
    }
  }
  hm = block_max<NW>(hm, red, 0);
  sm = block_max<NW>(sm, red, 1);
  h1 = block_sum<NW>(h1, red, 2);
  if (threadIdx.x == 0) {
    S->hinf = hm; S->stinf = sm; S->h1 = h1;
    if (!finite(hm) || !finite(sm)) {
      S->status = SNAP_ST_NONFINITE; S->phase = 2;
    } else if (hm <= A.opt.tol_h && sm <= A.opt.tol_s * S->uscale) {
      S->status = SNAP_ST_CONVERGED; S->phase = keep ? 1 : 2;
    } else if (S->iters >= A.opt.max_newton) {
      S->status = SNAP_ST_MAX_ITER; S->phase = 2;
    }
  }
}

// Schur factor with the fused forward substitution (also the final factor
// at the returned point when the adjoint will need it)
template <int BB, int NW, typename R>
SNAP_BAND_KERNEL void band_factor(KernelArgs A) {
  const int sid = A.order[blockIdx.x];
  const snap_sample_desc D = A.descs[sid];
  __shared__ BandShared<BB, NW, R> sh;
  const Ctx C = make_ctx(A, D, sid, false);
  const WsLayout WL = ws_layout(C.nx, C.nt, BB, sizeof(R));
  BandState* S = (BandState*)(C.ws + WL.hdr);
  const int phase = S->phase;
  if (phase == 2) return;
  // Local phase (||h||_inf <= kReuseH): S moves by O(||p||) between
  // iterations, so the previous iteration's factor, with float64 iterative
  // refinement against the current S (matrix free), solves the Newton system
  // to the same accuracy.  That pays where a factorization costs more than
  // the two or three substitution sweeps of the refinement: on the wide bands
  // (BB >= 13, Nx > 128), whose factorization chains are the longest of a
  // ragged batch; at BB <= 9 (measured on 512 samples of 128 x 128) a fresh
  // factorization is cheaper.
  if (BB >= 13 && phase == 0 && S->factored && S->hinf <= kReuseH) {
    assemble_rhs<NW>(C, WL);
    if (threadIdx.x == 0) S->reuse = 1;
    return;
  }
  if (threadIdx.x < 4) sh.flag[threadIdx.x] = 0;
  __syncthreads();
  assemble_all<NW>(C, WL);
  const int bad = factor_sweep<BB, NW, R>(C, WL, sh, make_part<BB>(C, kWhole));
  if (threadIdx.x == 0) {
    S->reuse = 0;
    S->factored = bad ? 0 : 1;
    if (phase == 1) {
      S->factor_ok = bad ? 0 : 1;
      S->phase = 2;
    } else if (bad) {
      S->status = SNAP_ST_SINGULAR_PIVOT;
      S->phase = 2;
    }
  }
}

// backward substitution (+ refinement in the mixed form): lam+ = lam + dlam
template <int BB, int NW, typename R>
SNAP_BAND_KERNEL void band_solve(KernelArgs A) {
  const int sid = A.order[blockIdx.x];
  const snap_sample_desc D = A.descs[sid];
  __shared__ BandShared<BB, NW, R> sh;
  const Ctx C = make_ctx(A, D, sid, false);
  const WsLayout WL = ws_layout(C.nx, C.nt, BB, sizeof(R));
  BandState* S = (BandState*)(C.ws + WL.hdr);
  if (S->phase != 0) return;
  double* lamp = (double*)(C.ws + WL.lamp);
  // Mixed form: the Newton iteration itself corrects the float32 solve (its
  // right-hand side h - J W^{-1} g is formed in float64 every iteration), so
  // explicit float64 refinement is applied only in the local phase, where the
  // float32 error would otherwise limit the last digits.
  const bool reuse = S->reuse != 0;
  const int max_ref = (S->hinf <= 1e-6 || reuse) ? 6 : 0;
  // a Newton step only needs its Schur residual well below the feasibility
  // tolerance (the next evaluation re-forms h in float64)
  const int refines = solve_with_factor<BB, NW, R>(C, WL, sh, !reuse, lamp, max_ref, 0.1 * A.opt.tol_h,
                                                   reuse);
  for (int r = threadIdx.x; r < C.m; r += NW * kWave) lamp[r] += C.lam[r];
  if (threadIdx.x == 0) S->refines += refines;
}

// x = L^{-T} D^{-1} y of a two-sided factor, the rows of one side: both
// sides first sweep the separator (the bottom keeps its rows out of xout),
// the bottom then turns the separator's x into its reversed coordinates
template <int BB, int NW, typename R>
__device__ __attribute__((always_inline)) void split_backward(const Ctx& C, const WsLayout& WL,
                                                              BandShared<BB, NW, R>& sh, int side, double* xout,
                                                              const double* addlam) {
  static_assert(NW * kWave >= BB * kT, "the separator's x is staged in part[]");
  const Part PT = make_part<BB>(C, kTop);
  const int K = PT.K, Kb = PT.Kb;
  const double* Y = (const double*)(C.ws + WL.Y);
  if (side == 0) {
    backward_sweep<BB, NW, R>(C, WL, sh, Y, xout, BackRange{K + BB - 1, 0, K + BB, false, false, true, addlam});
    return;
  }
  backward_sweep<BB, NW, R>(C, WL, sh, Y, xout, BackRange{K + BB - 1, K, K + BB, false, false, false, nullptr});
  for (int i = threadIdx.x; i < BB * kT; i += NW * kWave) {
    const int ib = i / kT, a = i - ib * kT;    // reversed local row ib, entry a
    sh.part[i] = sh.ring[((K + BB - 1 - ib) % (BB + 1)) * kT + (15 - a)];
  }
  __syncthreads();
  for (int i = threadIdx.x; i < (BB + 1) * kT; i += NW * kWave) {
    const int ib = i / kT, a = i - ib * kT;
    sh.ring[((Kb + ib) % (BB + 1)) * kT + a] = ib < BB ? sh.part[i] : 0.0;
  }
  __syncthreads();
  backward_sweep<BB, NW, R>(C, WL, sh, Y, xout, BackRange{Kb - 1, 0, Kb + BB, true, true, true, addlam});
}

// Solve S x = rin (internal order) with a two-sided factor in one
// workgroup: forward substitution of both sides and the separator, then the
// backward substitution of both sides (x canonical, every row written).
template <int BB, int NW, typename R>
__device__ __attribute__((always_inline)) void split_sweeps(const Ctx& C, const WsLayout& WL,
                                                            BandShared<BB, NW, R>& sh, double* x) {
  const double* rin = (const double*)(C.ws + WL.rin);
  double* Y = (double*)(C.ws + WL.Y);
  forward_sweep<BB, NW, R>(C, WL, sh, rin, Y, make_part<BB>(C, kTop));
  forward_sweep<BB, NW, R>(C, WL, sh, rin, Y, make_part<BB>(C, kBottom));
  forward_sweep<BB, NW, R>(C, WL, sh, rin, Y, make_part<BB>(C, kSep));
  split_backward<BB, NW, R>(C, WL, sh, 0, x, nullptr);
  split_backward<BB, NW, R>(C, WL, sh, 1, x, nullptr);
}

// Float64 iterative refinement of x (canonical) against rvec with a two-sided
// factor, in one workgroup: at most max_ref rounds, until the Schur residual
// (matrix free, float64) is below max(1e-13 ||rvec||, abs_floor).  Returns
// the rounds taken.  Uses res, rin and t as scratch.
template <int BB, int NW, typename R>
__device__ int split_refine(const Ctx& C, const WsLayout& WL, BandShared<BB, NW, R>& sh, double* x, int max_ref,
                            double abs_floor) {
  const double* rvec = (const double*)(C.ws + WL.rvec);
  double* res = (double*)(C.ws + WL.res);
  double* rin = (double*)(C.ws + WL.rin);
  double* dx = (double*)(C.ws + WL.t);
  double rn = 0.0;
  for (int r = threadIdx.x; r < C.m; r += NW * kWave) rn = fmax(rn, fabs(rvec[r]));
  rn = block_max<NW>(rn, sh.red, 1);
  int refines = 0;
  for (int it = 0; it < max_ref; ++it) {
    const double rm = schur_residual<NW>(C, WL, x, res, sh.red);
    if (!(rm > fmax(1e-13 * rn, abs_floor))) break;
    to_internal<NW>(C, res, rin);
    split_sweeps<BB, NW, R>(C, WL, sh, dx);
    for (int r = threadIdx.x; r < C.m; r += NW * kWave) x[r] += dx[r];
    __syncthreads();
    ++refines;
  }
  return refines;
}

// h of row (k, x) at u + alpha p
__device__ __forceinline__ double h_trial(const Ctx& C, const double* pv, double alpha, int k, int x) {
  const size_t b0 = (size_t)k * C.nx;
  const int xp = wrap(x + 1, C.nx), xm = wrap(x - 1, C.nx);
  const double u0 = C.u[b0 + x] + alpha * pv[b0 + x];
  const double up = C.u[b0 + xp] + alpha * pv[b0 + xp];
  const double um = C.u[b0 + xm] + alpha * pv[b0 + xm];
  const double un = C.u[b0 + C.nx + x] + alpha * pv[b0 + C.nx + x];
  return h_of(C, um, u0, up, un);
}

// ||h||_1 at u + alpha p
template <int NW>
__device__ double h1_trial(const Ctx& C, const double* pv, double alpha, double (*red)[4]) {
  double ht = 0.0;
  for (int r = threadIdx.x; r < C.m; r += NW * kWave) {
    const int k = r / C.nx, x = r - k * C.nx;
    ht += fabs(h_trial(C, pv, alpha, k, x));
  }
  return block_sum<NW>(ht, red, 1);
}

// Armijo backtracking of the l1 merit phi = 1/2||u - u_hat||^2 + mu ||h||_1
// along p: trial steps alpha, alpha/2, ... (ntries of them).  Its change is
// formed from differences (alpha d.p + alpha^2/2 p.p + mu (||h_t||_1 -
// ||h||_1)), never from phi values themselves, so rounding of the large sums
// cancels.  Returns the accepted step, or 0; counts the rejected trials.
// With soc_stop, a rejected full step that raised ||h||_1 stops the search
// (soc is set) for a second-order correction.
template <int NW>
__device__ double merit_search(const Ctx& C, const double* pv, double dd, double pp, double mu, double h1,
                               double hinf, double alpha, int ntries, double (*red)[4], int& backtracks,
                               bool soc_stop, bool& soc) {
  const double dphi = dd - mu * h1;
  soc = false;
  for (int i = 0; i < ntries; ++i) {
    const double ht = h1_trial<NW>(C, pv, alpha, red);
    const double dphi_t = alpha * dd + 0.5 * alpha * alpha * pp + mu * (ht - h1);
    // local phase (||h||_inf <= 1e-6): full Newton steps; there the change of
    // ||h||_1 along p sits below the rounding of the row sums
    // (with W >= 0.1 the step is a descent direction of the merit unless it
    // is zero; a zero step is taken, any other step must pass the test)
    if (dphi_t <= 1e-4 * alpha * dphi || !(pp > 0.0) || hinf <= 1e-6) return alpha;
    ++backtracks;
    if (i == 0 && soc_stop && ht > h1) {
      soc = true;
      return 0.0;
    }
    alpha *= 0.5;
  }
  return 0.0;
}

// step p = -W^{-1}(u - u_hat + J^T lam+), l1-merit backtracking, update
template <int BB, int NW, typename R>
SNAP_BAND_KERNEL void band_step(KernelArgs A) {
  const int sid = A.order[blockIdx.x];
  const snap_sample_desc D = A.descs[sid];
  __shared__ double red[NW][4];
  const Ctx C = make_ctx(A, D, sid, false);
  const WsLayout WL = ws_layout(C.nx, C.nt, BB, sizeof(R));
  BandState* S = (BandState*)(C.ws + WL.hdr);
  if (S->phase != 0) return;
  const int NT = NW * kWave;
  const double* lamp = (const double*)(C.ws + WL.lamp);
  double* pv = (double*)(C.ws + WL.p);
  double dd = 0.0, pp = 0.0, lmax = 0.0;
  for (int v = threadIdx.x; v < C.n; v += NT) {
    const int k = v / C.nx, x = v - k * C.nx;
    const double d = dres(C, v);
    const double p = -(d + jt_at(C, lamp, k, x)) / w_at(C, k, x);
    pv[v] = p;
    dd += d * p;
    pp += p * p;
  }
  for (int r = threadIdx.x; r < C.m; r += NT) lmax = fmax(lmax, fabs(lamp[r]));
  dd = block_sum<NW>(dd, red, 0);
  pp = block_sum<NW>(pp, red, 2);
  lmax = block_max<NW>(lmax, red, 1);
  const double h1 = S->h1, hinf = S->hinf;
  const double mu = fmax(S->mu, 1.1 * lmax + 1e-8);
  int backtracks = 0;
  bool soc = false;
  const bool soc_on = (A.opt.flags & SNAP_FLAG_SOC) != 0;
  const double alpha =
      merit_search<NW>(C, pv, dd, pp, mu, h1, hinf, 1.0, A.opt.max_ls + 1, red, backtracks, soc_on, soc);
  if (soc) {
    // band_soc tries u + p + p_soc, then halves along p
    if (threadIdx.x == 0) {
      S->mu = mu;
      S->backtracks += backtracks;
      S->soc_try = 1;
      S->soc_dd = dd;
      S->soc_pp = pp;
    }
    return;
  }
  const int ok = alpha > 0.0;
  if (ok) {
    for (int v = threadIdx.x; v < C.n; v += NT) C.u[v] += alpha * pv[v];
    for (int r = threadIdx.x; r < C.m; r += NT) C.lam[r] += alpha * (lamp[r] - C.lam[r]);
  }
  if (threadIdx.x == 0) {
    S->mu = mu;
    S->backtracks += backtracks;
    S->soc_try = 0;
    if (ok) {
      S->iters += 1;
    } else {
      S->status = SNAP_ST_LS_FAIL;
      S->phase = 2;
    }
  }
}

// Second-order correction (SNAP_FLAG_SOC), after band_step rejected the full
// step and it raised ||h||_1: with the step's factor (one- or two-sided,
// swept here by one workgroup), solve S z = h(u + p) and try
// u + q, q = p - W^{-1} J^T z, under the same Armijo test (the directional
// derivative of p); if it fails, halve along p from alpha = 1/2.
template <int BB, int NW, typename R, bool SPLIT>
SNAP_BAND_KERNEL void band_soc(KernelArgs A) {
  const int sid = A.order[blockIdx.x];
  const snap_sample_desc D = A.descs[sid];
  __shared__ BandShared<BB, NW, R> sh;
  const Ctx C = make_ctx(A, D, sid, false);
  const WsLayout WL = ws_layout(C.nx, C.nt, BB, sizeof(R));
  BandState* S = (BandState*)(C.ws + WL.hdr);
  if (S->phase != 0 || !S->soc_try) return;
  const int NT = NW * kWave;
  const double* pv = (const double*)(C.ws + WL.p);
  const double* lamp = (const double*)(C.ws + WL.lamp);
  double* rin = (double*)(C.ws + WL.rin);
  double* rvec = (double*)(C.ws + WL.rvec);
  double* z = (double*)(C.ws + WL.z);
  double* qv = (double*)(C.ws + WL.t);
  for (int r = threadIdx.x; r < C.M; r += NT) {
    double v = 0.0;
    if (r < C.m) {
      const int k = r / C.nx, px = r - k * C.nx, x = fold_x(px, C.nx);
      v = h_trial(C, pv, 1.0, k, x);
      rvec[(size_t)k * C.nx + x] = v;
    }
    rin[r] = v;
  }
  __syncthreads();
  if constexpr (SPLIT) {
    split_sweeps<BB, NW, R>(C, WL, sh, z);
    if (sizeof(R) == 4) (void)split_refine<BB, NW, R>(C, WL, sh, z, 6, 0.1 * A.opt.tol_h);
  } else {
    (void)solve_with_factor<BB, NW, R>(C, WL, sh, false, z, 6, 0.1 * A.opt.tol_h, false);
  }
  double dq = 0.0, qq = 0.0;
  for (int v = threadIdx.x; v < C.n; v += NT) {
    const int k = v / C.nx, x = v - k * C.nx;
    const double q = pv[v] - jt_at(C, z, k, x) / w_at(C, k, x);
    qv[v] = q;
    dq += dres(C, v) * q;
    qq += q * q;
  }
  dq = block_sum<NW>(dq, sh.red, 0);
  qq = block_sum<NW>(qq, sh.red, 2);
  const double mu = S->mu, h1 = S->h1, hinf = S->hinf, dd = S->soc_dd, pp = S->soc_pp;
  const double ht = h1_trial<NW>(C, qv, 1.0, sh.red);
  int backtracks = 0, taken = 0;
  double alpha = 0.0;
  if (dq + 0.5 * qq + mu * (ht - h1) <= 1e-4 * (dd - mu * h1)) {
    for (int v = threadIdx.x; v < C.n; v += NT) C.u[v] += qv[v];
    for (int r = threadIdx.x; r < C.m; r += NT) C.lam[r] = lamp[r];
    taken = 1;
  } else {
    bool soc = false;
    alpha = merit_search<NW>(C, pv, dd, pp, mu, h1, hinf, 0.5, A.opt.max_ls, sh.red, backtracks, false, soc);
    if (alpha > 0.0) {
      for (int v = threadIdx.x; v < C.n; v += NT) C.u[v] += alpha * pv[v];
      for (int r = threadIdx.x; r < C.m; r += NT) C.lam[r] += alpha * (lamp[r] - C.lam[r]);
      taken = 1;
    }
  }
  if (threadIdx.x == 0) {
    S->soc_try = 0;
    S->backtracks += backtracks;
    if (taken) {
      S->iters += 1;
    } else {
      S->status = SNAP_ST_LS_FAIL;
      S->phase = 2;
    }
  }
}

// per-sample statistics
template <int BB, int NW, typename R>
SNAP_BAND_KERNEL void band_finish(KernelArgs A) {
  const int sid = A.order[blockIdx.x];
  const snap_sample_desc D = A.descs[sid];
  const Ctx C = make_ctx(A, D, sid, false);
  const WsLayout WL = ws_layout(C.nx, C.nt, BB, sizeof(R));
  const BandState* S = (const BandState*)(C.ws + WL.hdr);
  if (threadIdx.x == 0) {
    snap_sample_stats st;
    st.status = S->status;
    st.newton_iters = S->iters;
    st.ls_backtracks = S->backtracks;
    st.refine_steps = S->refines;
    st.h_inf = S->hinf;
    st.stat_inf = S->stinf;
    A.stats[sid] = st;
  }
}

// adjoint right-hand side J W^{-1} g of rows [r0, r1) (internal order; rvec too)
template <int NW>
__device__ void adjoint_rhs_rows(const Ctx& C, const WsLayout& WL, int r0, int r1) {
  double* rin = (double*)(C.ws + WL.rin);
  double* rvec = (double*)(C.ws + WL.rvec);
  for (int r = r0 + (int)threadIdx.x; r < r1; r += NW * kWave) {
    double v = 0.0;
    if (r < C.m) {
      const int k = r / C.nx, px = r - k * C.nx, x = fold_x(px, C.nx);
      const int xp = wrap(x + 1, C.nx), xm = wrap(x - 1, C.nx);
      const double* U = C.u + (size_t)k * C.nx;
      double s = C.g[(size_t)(k + 1) * C.nx + x] / w_at(C, k + 1, x);
      if (C.god) {
        const GRow g = grow(C, U, x);
        s += g.c0 * C.g[(size_t)k * C.nx + x] / w_at(C, k, x);
        s += g.cr * C.g[(size_t)k * C.nx + xp] / w_at(C, k, xp);
        s += g.cl * C.g[(size_t)k * C.nx + xm] / w_at(C, k, xm);
      } else {
        s += C.cd * C.g[(size_t)k * C.nx + x] / w_at(C, k, x);
        s += (C.q * U[xp] - C.c) * C.g[(size_t)k * C.nx + xp] / w_at(C, k, xp);
        s += (-C.q * U[xm] - C.c) * C.g[(size_t)k * C.nx + xm] / w_at(C, k, xm);
      }
      v = s;
      rvec[(size_t)k * C.nx + x] = s;
    }
    rin[r] = v;
  }
  __syncthreads();
}

// grad = W^{-1}(g - J^T b) from b (canonical order) and the sample's statistics
template <int NW>
__device__ void adjoint_finish(const KernelArgs& A, const Ctx& C, const snap_sample_desc& D, int sid,
                               const double* lamp, int bad, int refines) {
  int floored = 0;
  for (int v = threadIdx.x; v < C.n; v += NW * kWave) {
    const int k = v / C.nx, x = v - k * C.nx;
    A.grad_uhat[D.var_off + v] = (C.g[v] - jt_at(C, lamp, k, x)) / w_at(C, k, x);
    if (k <= C.nt - 2) floored |= w_raw(C, k, x) < kWFloor;
  }
  floored = __syncthreads_or(floored);
  if (threadIdx.x == 0) {
    snap_sample_stats st;
    st.status = bad ? SNAP_ST_SINGULAR_PIVOT : (floored ? SNAP_ST_HESSIAN_FLOOR : SNAP_ST_CONVERGED);
    st.newton_iters = 0; st.ls_backtracks = 0; st.refine_steps = refines;
    st.h_inf = 0.0; st.stat_inf = 0.0;
    A.stats[sid] = st;
  }
}

// adjoint: S b = J W^{-1} g, grad = W^{-1}(g - J^T b), at (u*, lam*); reuses
// the factor when the forward kept one at this point, else factors here
template <int BB, int NW, typename R>
SNAP_BAND_KERNEL void band_adjoint(KernelArgs A) {
  const int sid = A.order[blockIdx.x];
  const snap_sample_desc D = A.descs[sid];
  __shared__ BandShared<BB, NW, R> sh;
  const Ctx C = make_ctx(A, D, sid, true);
  const WsLayout WL = ws_layout(C.nx, C.nt, BB, sizeof(R));
  const BandState* S = (const BandState*)(C.ws + WL.hdr);
  double* lamp = (double*)(C.ws + WL.lamp);
  const bool keep = (A.opt.flags & SNAP_FLAG_KEEP_FACTOR) != 0;
  const bool have = keep && S->factor_ok == 1;
  if (threadIdx.x < 4) sh.flag[threadIdx.x] = 0;
  __syncthreads();
  int bad = 0;
  if (have) {
    adjoint_rhs_rows<NW>(C, WL, 0, C.M);
  } else {
    assemble_all<NW>(C, WL);
    bad = factor_sweep<BB, NW, R>(C, WL, sh, make_part<BB>(C, kWhole));
  }
  const int refines = solve_with_factor<BB, NW, R>(C, WL, sh, !have, lamp);
  adjoint_finish<NW>(A, C, D, sid, lamp, bad, refines);
}

// ------------------------------------------------------------------ two-sided form
// Kernels of the two-sided factorization (see the parts section): launches
// marked "two per sample" run the top part in workgroup 2i and the bottom
// part in workgroup 2i + 1 of sample order[i]; the separator kernels run one
// workgroup per sample.  With a float32 factor the float64 refinement rounds
// (the local phase of the Newton solve, the adjoint) run in one workgroup per
// sample over all three parts of the factor.

// rows of a side: the top assembles block rows [0, K + BB), the bottom
// [K + BB, NB) and its own copy of the separator rows (no right-hand side)
template <int NW>
__device__ void assemble_part(const Ctx& C, const WsLayout& WL, const Part& P) {
  int* acol = (int*)(C.ws + WL.acol);
  double* aval = (double*)(C.ws + WL.aval);
  const int s0 = P.K * kT, s1 = (C.NB - P.Kb) * kT;
  if (P.kind == kTop) {
    assemble_rows<NW>(C, WL, 0, s1, acol, aval, 0, true);
  } else {
    assemble_rows<NW>(C, WL, s1, C.M, acol, aval, 0, true);
    assemble_rows<NW>(C, WL, s0, s1, (int*)(C.ws + WL.scol), (double*)(C.ws + WL.sval), s0, false);
  }
}

// (two per sample) factor a side at the current (u, lam), fused forward
// substitution, export of the side's separator update
template <int BB, int NW, typename R>
SNAP_BAND_KERNEL void band_split_factor(KernelArgs A) {
  const int side = blockIdx.x & 1;
  const int sid = A.order[blockIdx.x >> 1];
  const snap_sample_desc D = A.descs[sid];
  __shared__ BandShared<BB, NW, R> sh;
  const Ctx C = make_ctx(A, D, sid, false);
  const WsLayout WL = ws_layout(C.nx, C.nt, BB, sizeof(R));
  BandState* S = (BandState*)(C.ws + WL.hdr);
  // (a reused factor: band_split_rhs did this step's work; the final factor
  // at the returned point, phase 1, is always taken)
  if (S->phase == 2 || (S->phase == 0 && S->reuse)) return;
  const Part PT = make_part<BB>(C, side ? kBottom : kTop);
  assemble_part<NW>(C, WL, PT);
  if (threadIdx.x < 4) sh.flag[threadIdx.x] = 0;
  __syncthreads();
  const int bad = factor_sweep<BB, NW, R>(C, WL, sh, PT);
  if (threadIdx.x == 0) S->side_bad[side] = bad;
}

// (two per sample) Local phase (||h||_inf <= kReuseH): the step is solved
// with the previous iteration's factor and float64 refinement, as on
// one-sided wide bands.  Decides that (the top workgroup sets the flag; no
// other workgroup of this launch reads it), and then forms the side's
// right-hand side and its forward substitution in place of the
// factorization.
template <int BB, int NW, typename R>
SNAP_BAND_KERNEL void band_split_rhs(KernelArgs A) {
  const int side = blockIdx.x & 1;
  const int sid = A.order[blockIdx.x >> 1];
  const snap_sample_desc D = A.descs[sid];
  __shared__ BandShared<BB, NW, R> sh;
  const Ctx C = make_ctx(A, D, sid, false);
  const WsLayout WL = ws_layout(C.nx, C.nt, BB, sizeof(R));
  BandState* S = (BandState*)(C.ws + WL.hdr);
  const int phase = S->phase;
  if (phase == 2) return;
  const bool reuse = phase == 0 && S->factored && S->hinf <= kReuseH;
  if (threadIdx.x == 0 && side == 0) S->reuse = reuse ? 1 : 0;
  if (!reuse) return;
  const Part PT = make_part<BB>(C, side ? kBottom : kTop);
  const int s1 = (C.NB - PT.Kb) * kT;
  assemble_rhs_rows<NW>(C, WL, side ? s1 : 0, side ? C.M : s1);
  forward_sweep<BB, NW, R>(C, WL, sh, (const double*)(C.ws + WL.rin), (double*)(C.ws + WL.Y), PT);
}

// (one per sample) factor the separator; the state update of band_factor
template <int BB, int NW, typename R>
SNAP_BAND_KERNEL void band_split_sep(KernelArgs A) {
  const int sid = A.order[blockIdx.x];
  const snap_sample_desc D = A.descs[sid];
  __shared__ BandShared<BB, NW, R> sh;
  const Ctx C = make_ctx(A, D, sid, false);
  const WsLayout WL = ws_layout(C.nx, C.nt, BB, sizeof(R));
  BandState* S = (BandState*)(C.ws + WL.hdr);
  const int phase = S->phase;
  if (phase == 2) return;
  if (phase == 0 && S->reuse) {
    // the separator's forward substitution with the stored factor
    forward_sweep<BB, NW, R>(C, WL, sh, (const double*)(C.ws + WL.rin), (double*)(C.ws + WL.Y),
                             make_part<BB>(C, kSep));
    return;
  }
  if (threadIdx.x < 4) sh.flag[threadIdx.x] = 0;
  __syncthreads();
  const int bad = factor_sweep<BB, NW, R>(C, WL, sh, make_part<BB>(C, kSep)) | S->side_bad[0] | S->side_bad[1];
  if (threadIdx.x == 0) {
    S->reuse = 0;
    S->factored = bad ? 0 : 1;
    if (phase == 1) {
      S->factor_ok = bad ? 0 : 1;
      S->phase = 2;
    } else if (bad) {
      S->status = SNAP_ST_SINGULAR_PIVOT;
      S->phase = 2;
    }
  }
}

// (two per sample) backward substitution: lam+ = lam + dlam, a side's rows
template <int BB, int NW, typename R>
SNAP_BAND_KERNEL void band_split_solve(KernelArgs A) {
  const int side = blockIdx.x & 1;
  const int sid = A.order[blockIdx.x >> 1];
  const snap_sample_desc D = A.descs[sid];
  __shared__ BandShared<BB, NW, R> sh;
  const Ctx C = make_ctx(A, D, sid, false);
  const WsLayout WL = ws_layout(C.nx, C.nt, BB, sizeof(R));
  const BandState* S = (const BandState*)(C.ws + WL.hdr);
  if (S->phase != 0) return;
  // float64 with a fresh factor: lam+ = lam + dlam directly; a float32 or
  // reused factor: dlam to z, refined and added by band_split_refine
  if (sizeof(R) == 8 && !S->reuse)
    split_backward<BB, NW, R>(C, WL, sh, side, (double*)(C.ws + WL.lamp), C.lam);
  else
    split_backward<BB, NW, R>(C, WL, sh, side, (double*)(C.ws + WL.z), nullptr);
}

// A refinement round of the two-sided step, spread over the solve's
// launches: band_split_res (one per sample) decides it and forms the
// internal-order residual; band_split_rfwd (two per sample) and
// band_split_rsep (one) run the forward substitution; band_split_rbwd (two)
// the backward substitution, adding the correction to dlam (z).  Rounds
// still due after it are swept by band_split_refine in one workgroup.
template <int BB, int NW, typename R>
__device__ __forceinline__ bool split_refining(const BandState* S) {
  return S->phase == 0 && ((sizeof(R) == 4 && S->hinf <= 1e-6) || S->reuse);
}

template <int BB, int NW, typename R>
SNAP_BAND_KERNEL void band_split_res(KernelArgs A) {
  const int sid = A.order[blockIdx.x];
  const snap_sample_desc D = A.descs[sid];
  __shared__ double red[NW][4];
  const Ctx C = make_ctx(A, D, sid, false);
  const WsLayout WL = ws_layout(C.nx, C.nt, BB, sizeof(R));
  BandState* S = (BandState*)(C.ws + WL.hdr);
  if (S->phase == 2) return;
  int round = 0;
  if (split_refining<BB, NW, R>(S)) {
    const double* rvec = (const double*)(C.ws + WL.rvec);
    double* res = (double*)(C.ws + WL.res);
    double rn = 0.0;
    for (int r = threadIdx.x; r < C.m; r += NW * kWave) rn = fmax(rn, fabs(rvec[r]));
    rn = block_max<NW>(rn, red, 1);
    const double rm = schur_residual<NW>(C, WL, (const double*)(C.ws + WL.z), res, red);
    if (rm > fmax(1e-13 * rn, 0.1 * A.opt.tol_h)) {
      to_internal<NW>(C, res, (double*)(C.ws + WL.rin));
      round = 1;
    }
  }
  if (threadIdx.x == 0) {
    S->round = round;
    if (round) S->refines += 1;
  }
}

template <int BB, int NW, typename R>
SNAP_BAND_KERNEL void band_split_rfwd(KernelArgs A) {
  const int side = blockIdx.x & 1;
  const int sid = A.order[blockIdx.x >> 1];
  const snap_sample_desc D = A.descs[sid];
  __shared__ BandShared<BB, NW, R> sh;
  const Ctx C = make_ctx(A, D, sid, false);
  const WsLayout WL = ws_layout(C.nx, C.nt, BB, sizeof(R));
  const BandState* S = (const BandState*)(C.ws + WL.hdr);
  if (S->phase != 0 || !S->round) return;
  forward_sweep<BB, NW, R>(C, WL, sh, (const double*)(C.ws + WL.rin), (double*)(C.ws + WL.Y),
                           make_part<BB>(C, side ? kBottom : kTop));
}

template <int BB, int NW, typename R>
SNAP_BAND_KERNEL void band_split_rsep(KernelArgs A) {
  const int sid = A.order[blockIdx.x];
  const snap_sample_desc D = A.descs[sid];
  __shared__ BandShared<BB, NW, R> sh;
  const Ctx C = make_ctx(A, D, sid, false);
  const WsLayout WL = ws_layout(C.nx, C.nt, BB, sizeof(R));
  const BandState* S = (const BandState*)(C.ws + WL.hdr);
  if (S->phase != 0 || !S->round) return;
  forward_sweep<BB, NW, R>(C, WL, sh, (const double*)(C.ws + WL.rin), (double*)(C.ws + WL.Y),
                           make_part<BB>(C, kSep));
}

template <int BB, int NW, typename R>
SNAP_BAND_KERNEL void band_split_rbwd(KernelArgs A) {
  const int side = blockIdx.x & 1;
  const int sid = A.order[blockIdx.x >> 1];
  const snap_sample_desc D = A.descs[sid];
  __shared__ BandShared<BB, NW, R> sh;
  const Ctx C = make_ctx(A, D, sid, false);
  const WsLayout WL = ws_layout(C.nx, C.nt, BB, sizeof(R));
  const BandState* S = (const BandState*)(C.ws + WL.hdr);
  if (S->phase != 0 || !S->round) return;
  double* z = (double*)(C.ws + WL.z);
  split_backward<BB, NW, R>(C, WL, sh, side, z, z);     // z += correction
}

// (one per sample) float64 refinement of dlam, then lam+ = lam + dlam: with
// a float32 factor in the local phase (as the one-sided mixed solve), and
// with a reused factor; nothing with a fresh float64 factor
template <int BB, int NW, typename R>
SNAP_BAND_KERNEL void band_split_refine(KernelArgs A) {
  const int sid = A.order[blockIdx.x];
  const snap_sample_desc D = A.descs[sid];
  __shared__ BandShared<BB, NW, R> sh;
  const Ctx C = make_ctx(A, D, sid, false);
  const WsLayout WL = ws_layout(C.nx, C.nt, BB, sizeof(R));
  BandState* S = (BandState*)(C.ws + WL.hdr);
  if (S->phase != 0) return;
  const bool reuse = S->reuse != 0;
  if (sizeof(R) == 8 && !reuse) return;
  double* z = (double*)(C.ws + WL.z);
  double* lamp = (double*)(C.ws + WL.lamp);
  const int refines =
      (S->hinf <= 1e-6 || reuse) ? split_refine<BB, NW, R>(C, WL, sh, z, 6, 0.1 * A.opt.tol_h) : 0;
  for (int r = threadIdx.x; r < C.m; r += NW * kWave) lamp[r] = C.lam[r] + z[r];
  if (threadIdx.x == 0) S->refines += refines;
}

// adjoint, (two per sample): a side's right-hand side and forward
// substitution with the kept factor, or a side's factorization
template <int BB, int NW, typename R>
SNAP_BAND_KERNEL void band_split_adj1(KernelArgs A) {
  const int side = blockIdx.x & 1;
  const int sid = A.order[blockIdx.x >> 1];
  const snap_sample_desc D = A.descs[sid];
  __shared__ BandShared<BB, NW, R> sh;
  const Ctx C = make_ctx(A, D, sid, true);
  const WsLayout WL = ws_layout(C.nx, C.nt, BB, sizeof(R));
  BandState* S = (BandState*)(C.ws + WL.hdr);
  const bool have = (A.opt.flags & SNAP_FLAG_KEEP_FACTOR) != 0 && S->factor_ok == 1;
  const Part PT = make_part<BB>(C, side ? kBottom : kTop);
  if (have) {
    const int s1 = (C.NB - PT.Kb) * kT;
    adjoint_rhs_rows<NW>(C, WL, side ? s1 : 0, side ? C.M : s1);
    forward_sweep<BB, NW, R>(C, WL, sh, (const double*)(C.ws + WL.rin), (double*)(C.ws + WL.Y), PT);
  } else {
    assemble_part<NW>(C, WL, PT);
    if (threadIdx.x < 4) sh.flag[threadIdx.x] = 0;
    __syncthreads();
    const int bad = factor_sweep<BB, NW, R>(C, WL, sh, PT);
    if (threadIdx.x == 0) S->side_bad[side] = bad;
  }
}

// adjoint, (one per sample): the separator's forward substitution, or its
// factorization
template <int BB, int NW, typename R>
SNAP_BAND_KERNEL void band_split_adj2(KernelArgs A) {
  const int sid = A.order[blockIdx.x];
  const snap_sample_desc D = A.descs[sid];
  __shared__ BandShared<BB, NW, R> sh;
  const Ctx C = make_ctx(A, D, sid, true);
  const WsLayout WL = ws_layout(C.nx, C.nt, BB, sizeof(R));
  BandState* S = (BandState*)(C.ws + WL.hdr);
  const bool have = (A.opt.flags & SNAP_FLAG_KEEP_FACTOR) != 0 && S->factor_ok == 1;
  if (have) {
    forward_sweep<BB, NW, R>(C, WL, sh, (const double*)(C.ws + WL.rin), (double*)(C.ws + WL.Y),
                             make_part<BB>(C, kSep));
  } else {
    if (threadIdx.x < 4) sh.flag[threadIdx.x] = 0;
    __syncthreads();
    const int bad = factor_sweep<BB, NW, R>(C, WL, sh, make_part<BB>(C, kSep)) | S->side_bad[0] | S->side_bad[1];
    if (threadIdx.x == 0) S->adj_bad = bad;
  }
}

// adjoint, (two per sample): backward substitution, a side's rows of b
template <int BB, int NW, typename R>
SNAP_BAND_KERNEL void band_split_adj3(KernelArgs A) {
  const int side = blockIdx.x & 1;
  const int sid = A.order[blockIdx.x >> 1];
  const snap_sample_desc D = A.descs[sid];
  __shared__ BandShared<BB, NW, R> sh;
  const Ctx C = make_ctx(A, D, sid, true);
  const WsLayout WL = ws_layout(C.nx, C.nt, BB, sizeof(R));
  split_backward<BB, NW, R>(C, WL, sh, side, (double*)(C.ws + WL.lamp), nullptr);
}

// adjoint, (one per sample): the gradient and the statistics
template <int BB, int NW, typename R>
SNAP_BAND_KERNEL void band_split_adj4(KernelArgs A) {
  const int sid = A.order[blockIdx.x];
  const snap_sample_desc D = A.descs[sid];
  const Ctx C = make_ctx(A, D, sid, true);
  const WsLayout WL = ws_layout(C.nx, C.nt, BB, sizeof(R));
  const BandState* S = (const BandState*)(C.ws + WL.hdr);
  const bool have = (A.opt.flags & SNAP_FLAG_KEEP_FACTOR) != 0 && S->factor_ok == 1;
  double* b = (double*)(C.ws + WL.lamp);
  int refines = 0;
  if constexpr (sizeof(R) == 4) {
    // float32 factor: refine b to working precision, as the one-sided adjoint
    __shared__ BandShared<BB, NW, R> sh;
    refines = split_refine<BB, NW, R>(C, WL, sh, b, 6, 0.0);
  }
  adjoint_finish<NW>(A, C, D, sid, b, have ? 0 : S->adj_bad, refines);
}

// ------------------------------------------------------------------ dispatch
static const int kBBs[] = {1, 2, 3, 5, 7, 9, 13, 17};

static int pick_bb(int need) {
  for (int b : kBBs)
    if (b >= need) return b;
  return -1;
}

// Launch shape: NW wavefronts share one sample's block window.  Four let two
// samples run per CU; eight halve each wavefront's share of the trailing
// update.  Which wins depends on the batch, so both are built for BB <= 9 and
// the plan's autotuner picks (wider bands always take eight).
template <int BB, int NW, typename R>
static void launch_band(const KernelArgs& a, hipStream_t st) {
  const dim3 grid(a.count), block(NW * kWave);
  if (a.backward) {
    hipLaunchKernelGGL((band_adjoint<BB, NW, R>), grid, block, 0, st, a);
    return;
  }
  hipLaunchKernelGGL((band_init<BB, NW, R>), grid, block, 0, st, a);
  hipLaunchKernelGGL((band_eval<BB, NW, R>), grid, block, 0, st, a);
  KernelTimer* tm = tl_timer;
  for (int it = 0; it < a.opt.max_newton; ++it) {
    if (tm) timer_mark(tm, kTimedBandFactor, st);
    hipLaunchKernelGGL((band_factor<BB, NW, R>), grid, block, 0, st, a);
    if (tm) timer_mark(tm, kTimedBandFactor, st);
    if (tm) timer_mark(tm, kTimedBandSolve, st);
    hipLaunchKernelGGL((band_solve<BB, NW, R>), grid, block, 0, st, a);
    if (tm) timer_mark(tm, kTimedBandSolve, st);
    hipLaunchKernelGGL((band_step<BB, NW, R>), grid, block, 0, st, a);
    if (a.opt.flags & SNAP_FLAG_SOC) hipLaunchKernelGGL((band_soc<BB, NW, R, false>), grid, block, 0, st, a);
    hipLaunchKernelGGL((band_eval<BB, NW, R>), grid, block, 0, st, a);
  }
  // the final factor of a sample that converged at the last evaluation
  if (a.opt.flags & SNAP_FLAG_KEEP_FACTOR)
    hipLaunchKernelGGL((band_factor<BB, NW, R>), grid, block, 0, st, a);
  hipLaunchKernelGGL((band_finish<BB, NW, R>), grid, block, 0, st, a);
}

// the two-sided form: the same Newton loop with each factorization and
// backward substitution split over two workgroups per sample (see the parts
// section) and the separator's factorization in a launch of its own
template <int BB, int NW, typename R>
static void launch_band_split(const KernelArgs& a, hipStream_t st) {
  const dim3 one(a.count), two(2 * a.count), block(NW * kWave);
  if (a.backward) {
    hipLaunchKernelGGL((band_split_adj1<BB, NW, R>), two, block, 0, st, a);
    hipLaunchKernelGGL((band_split_adj2<BB, NW, R>), one, block, 0, st, a);
    hipLaunchKernelGGL((band_split_adj3<BB, NW, R>), two, block, 0, st, a);
    hipLaunchKernelGGL((band_split_adj4<BB, NW, R>), one, block, 0, st, a);
    return;
  }
  hipLaunchKernelGGL((band_init<BB, NW, R>), one, block, 0, st, a);
  hipLaunchKernelGGL((band_eval<BB, NW, R>), one, block, 0, st, a);
  KernelTimer* tm = tl_timer;
  for (int it = 0; it < a.opt.max_newton; ++it) {
    if (tm) timer_mark(tm, kTimedBandFactor, st);
    hipLaunchKernelGGL((band_split_rhs<BB, NW, R>), two, block, 0, st, a);
    hipLaunchKernelGGL((band_split_factor<BB, NW, R>), two, block, 0, st, a);
    hipLaunchKernelGGL((band_split_sep<BB, NW, R>), one, block, 0, st, a);
    if (tm) timer_mark(tm, kTimedBandFactor, st);
    if (tm) timer_mark(tm, kTimedBandSolve, st);
    hipLaunchKernelGGL((band_split_solve<BB, NW, R>), two, block, 0, st, a);
    hipLaunchKernelGGL((band_split_res<BB, NW, R>), one, block, 0, st, a);
    hipLaunchKernelGGL((band_split_rfwd<BB, NW, R>), two, block, 0, st, a);
    hipLaunchKernelGGL((band_split_rsep<BB, NW, R>), one, block, 0, st, a);
    hipLaunchKernelGGL((band_split_rbwd<BB, NW, R>), two, block, 0, st, a);
    hipLaunchKernelGGL((band_split_refine<BB, NW, R>), one, block, 0, st, a);
    if (tm) timer_mark(tm, kTimedBandSolve, st);
    hipLaunchKernelGGL((band_step<BB, NW, R>), one, block, 0, st, a);
    if (a.opt.flags & SNAP_FLAG_SOC) hipLaunchKernelGGL((band_soc<BB, NW, R, true>), one, block, 0, st, a);
    hipLaunchKernelGGL((band_eval<BB, NW, R>), one, block, 0, st, a);
  }
  if (a.opt.flags & SNAP_FLAG_KEEP_FACTOR) {
    hipLaunchKernelGGL((band_split_factor<BB, NW, R>), two, block, 0, st, a);
    hipLaunchKernelGGL((band_split_sep<BB, NW, R>), one, block, 0, st, a);
  }
  hipLaunchKernelGGL((band_finish<BB, NW, R>), one, block, 0, st, a);
}

// class = BB + kBandAlt * alt: alt 0 is the default launch shape (four
// wavefronts for BB <= 9, eight above), alt 1 the alternative (eight, BB <= 9),
// alt 2 the two-sided form (BB >= 13)
constexpr int kBandAlt = 32;
constexpr int kBandSplit = 2 * kBandAlt;

// The two-sided form halves a factorization's chain of panel steps at the
// cost of a third launch (the separator, BB panel steps) and twice the
// workgroups; it is the default where the chain is long (wide bands, at least
// 40 BB block rows).
static bool split_pays(int nx, int nt, int bb) {
  const int64_t m = (int64_t)nx * (nt - 1), nb = (m + kT - 1) / kT;
  return bb >= 13 && nb >= 40 * bb;
}

template <typename R>
static int launch_bb(int cls, const KernelArgs& a, hipStream_t st) {
  const int bb = cls % kBandAlt, alt = cls / kBandAlt;
#ifdef SNAP_BAND_QUICK
  if (bb <= SNAP_BAND_QUICK && alt == 0) {
    launch_band<SNAP_BAND_QUICK, (SNAP_BAND_QUICK <= 9 ? 4 : 8), R>(a, st);
    return hipGetLastError() == hipSuccess ? 0 : SNAP_EHIP;
  }
  return SNAP_EUNSUPPORTED;
#else
  if (alt == 0) {
    switch (bb) {
      case 1: launch_band<1, 4, R>(a, st); break;
      case 2: launch_band<2, 4, R>(a, st); break;
      case 3: launch_band<3, 4, R>(a, st); break;
      case 5: launch_band<5, 4, R>(a, st); break;
      case 7: launch_band<7, 4, R>(a, st); break;
      case 9: launch_band<9, 4, R>(a, st); break;
      case 13: launch_band<13, 8, R>(a, st); break;
      case 17: launch_band<17, 8, R>(a, st); break;
      default: return SNAP_EUNSUPPORTED;
    }
  } else if (alt == 1) {
    switch (bb) {
      case 1: launch_band<1, 8, R>(a, st); break;
      case 2: launch_band<2, 8, R>(a, st); break;
      case 3: launch_band<3, 8, R>(a, st); break;
      case 5: launch_band<5, 8, R>(a, st); break;
      case 7: launch_band<7, 8, R>(a, st); break;
      case 9: launch_band<9, 8, R>(a, st); break;
      default: return SNAP_EUNSUPPORTED;
    }
  } else if (alt == 2) {
    switch (bb) {
      case 13: launch_band_split<13, 8, R>(a, st); break;
      case 17: launch_band_split<17, 8, R>(a, st); break;
      default: return SNAP_EUNSUPPORTED;
    }
  } else {
    return SNAP_EUNSUPPORTED;
  }
  return hipGetLastError() == hipSuccess ? 0 : SNAP_EHIP;
#endif
}

bool band_supported(int nx, int nt, bool mixed) {
  (void)mixed;
  return nx >= 3 && nt >= 2 && pick_bb(band_bb(nx, nt)) > 0 && (int64_t)nx * nt < (1 << 30);
}

// Kernel class of a shape: the instantiated block half-bandwidth with the
// default launch shape, or its two-sided form where that pays.
int band_class(int nx, int nt, bool mixed) {
  if (!band_supported(nx, nt, mixed)) return -1;
  const int bb = pick_bb(band_bb(nx, nt));
  return split_pays(nx, nt, bb) ? bb + kBandSplit : bb;
}

// Classes the autotuner may choose between for a shape (default first): the
// other launch shape at BB <= 9; the one- or two-sided form above (the
// two-sided one where its parts have at least BB block rows each).
int band_variants(int nx, int nt, bool mixed, int* out, int cap) {
  const int cls = band_class(nx, nt, mixed);
  if (cls < 0 || cap < 1) return 0;
  const int bb = cls % kBandAlt;
  const int64_t nb = ((int64_t)nx * (nt - 1) + kT - 1) / kT;
  int n = 0;
  out[n++] = cls;
  if (n >= cap) return n;
  if (bb <= 9) {
    out[n++] = bb + kBandAlt;
  } else if (cls != bb) {
    out[n++] = bb;
  } else if (nb >= 3 * bb) {
    out[n++] = bb + kBandSplit;
  }
  return n;
}

// wavefronts per workgroup of a class (for plan descriptions)
int band_waves(int cls) { return (cls % kBandAlt) <= 9 && cls / kBandAlt == 0 ? 4 : 8; }

// workgroups per sample of a class's factorization
int band_sides(int cls) { return cls / kBandAlt == 2 ? 2 : 1; }

// The default class of a whole group: a group that leaves CUs idle (at most
// one sample per CU) takes the shape that puts more of a CU on each sample,
// eight wavefronts at BB <= 9, the two-sided factorization at BB >= 13
// (every sample's parts at least BB block rows).  min_nb is the fewest block
// rows of the group's samples.
int band_group_class(int cls, int min_nb, int count, int ncu) {
  const int bb = cls % kBandAlt;
  if (cls / kBandAlt != 0 || count > ncu) return cls;
  if (bb <= 9) return bb + kBandAlt;
  if (min_nb >= 3 * bb) return bb + kBandSplit;
  return cls;
}

size_t band_workspace_bytes(int nx, int nt, bool mixed) {  // the same for every launch shape
  const int bb = pick_bb(band_bb(nx, nt));
  return ws_layout(nx, nt, bb, mixed ? sizeof(float) : sizeof(double)).total;
}

int band_launch(const KernelArgs& a, int cls, bool mixed, hipStream_t st) {
  if (a.count == 0) return 0;
  return mixed ? launch_bb<float>(cls, a, st) : launch_bb<double>(cls, a, st);
}

}  // namespace snap
