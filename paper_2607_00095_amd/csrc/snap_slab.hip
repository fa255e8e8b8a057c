// Newton/SQP projection for the "slab-row" families: constraints that are
// global in x and local in time (paper Sec. III-A: mass-type rows touch one or
// two time slabs), plus initial-condition rows on slab 0.
//
//   SNAP_MASS_IC     rows sum_x u(.,k+1) - M0                   (k = 0..Nt-2)
//   SNAP_FISHER_KPP  rows sum_x u(.,k+1) - sum_x u(.,k) - dt*rho*sum_x u(.,k)(1-u(.,k))
//
// Both are written as row_k = sum_x u(x,k+1) + (terms in slab k), with
// a_k(x) = d row_k / d u(x,k) = -1 - c + 2c u(x,k), c = dt*rho (0 for mass
// rows).  The Hessian of lam^T h is diagonal and constant on a slab
// (2c*lam_k on slab k), so W = I + Hess(lam^T h) is one number W_k per slab.
//
// Schur form of the Newton-KKT system (Appendix B): with g = u - u_hat + J^T lam
// the stationarity residual, the multiplier increment solves
//     S dlam = h - J W^{-1} g,   S = J W^{-1} J^T,
// and the step is p = -W^{-1}(u - u_hat + J^T lam+), lam+ = lam + dlam.  With
// the IC rows first, S = [[D, C], [C^T, T]] with D_ii = 1/W_0,
// C_{i,0} = a_0(i)/W_0, T_kk = sum_x a_k^2/W_k + Nx/W_{k+1},
// T_{k,k+1} = sum_x a_{k+1}/W_{k+1}.  Eliminating the diagonal IC block cancels
// the slab-0 term of T_00 exactly, leaving a symmetric tridiagonal system in
// time, solved by parallel cyclic reduction inside one wavefront.  Because
// a_k is affine in u, four sums per slab (u, u^2, g, u*g) give every Schur
// entry and right-hand side.
//
// Layout.  One workgroup owns one sample for the whole Newton loop.  G
// consecutive lanes form a group that owns one time slab per round (round r
// covers slabs groups*r .. groups*(r+1)-1, the wavefronts' blocks of them
// rotated by one per round), lane `sub` of the group owns
// x = sub, sub+G, ...; the field u and the step p stay in registers and u_hat
// in LDS.  A slab sum is a log2(G)-step DPP scan inside the group, so every
// slab of a wavefront reduces at once.
//
// Iteration.  After wavefront 0 has solved for lam+, one pass over the field
// forms the step p and, at the trial point u + p with multipliers lam+, all
// four slab sums, the IC rows and the merit terms.  Wavefront 0 then decides
// the Armijo test of the l1 merit at alpha = 1 from those sums; on acceptance
// the same sums already describe the new iterate, so it goes straight on to
// the convergence test and the next solve.  Two workgroup barriers per Newton
// iteration; halving (alpha < 1) falls back to explicit trial passes.
#include "snap_device.hpp"

namespace snap {

int slab_wide_class(int nx, int nt);
int slab_wide_launch(const KernelArgs& a, int cls, bool mixed, hipStream_t st);

namespace {

constexpr int kMaxNt = 128;
constexpr double kWFloor = 0.1;

// compile-time tags: kinds of slab-sum pass (see the kernel), and flags
constexpr int kPoint = 0, kStep = 1;
template <int K>
struct PassKind {
  static constexpr int value = K;
};

// Value of v on lane addr/4 of the wavefront (ds_bpermute: the LDS
// crossbar without a memory round trip); every lane must be active.
template <typename TS>
__device__ __forceinline__ TS lane_get(TS v, int addr) {
  if constexpr (sizeof(TS) == 8) {
    const int lo = __builtin_amdgcn_ds_bpermute(addr, __double2loint(v));
    const int hi = __builtin_amdgcn_ds_bpermute(addr, __double2hiint(v));
    return __hiloint2double(hi, lo);
  } else {
    return __int_as_float(__builtin_amdgcn_ds_bpermute(addr, __float_as_int(v)));
  }
}

// Value of v on lane l-1 / l+1 (lane 0 / lane 63: its own), by DPP
// whole-wavefront shifts (wave_shr:1 / wave_shl:1): no LDS round trip.
template <typename TS, int CTRL>
__device__ __forceinline__ TS lane_shift(TS v) {
  if constexpr (sizeof(TS) == 8) {
    const int lo = __double2loint(v), hi = __double2hiint(v);
    return __hiloint2double(__builtin_amdgcn_update_dpp(hi, hi, CTRL, 0xf, 0xf, false),
                            __builtin_amdgcn_update_dpp(lo, lo, CTRL, 0xf, 0xf, false));
  } else {
    const int x = __float_as_int(v);
    return __int_as_float(__builtin_amdgcn_update_dpp(x, x, CTRL, 0xf, 0xf, false));
  }
}
template <typename TS> __device__ __forceinline__ TS lane_prev(TS v) { return lane_shift<TS, 0x138>(v); }
template <typename TS> __device__ __forceinline__ TS lane_next(TS v) { return lane_shift<TS, 0x130>(v); }

// Solve the symmetric tridiagonal system with diagonal Td[0..n),
// off-diagonal To[k] = T_{k,k+1} and right-hand side rhs by ONE wavefront
// (n <= 128), in precision TS; the result goes to x (LDS).  Lane l holds
// equations 2l and 2l+1.  One level of cyclic reduction eliminates the odd
// unknowns (each even equation takes its two odd neighbours), parallel cyclic
// reduction solves the <= 64 even equations, one per lane, and the odd
// unknowns follow by back-substitution.  One reciprocal per equation and level.
// Neighbours' coefficients move lane to lane by DPP shifts at distance 1
// and by ds_bpermute beyond.  No lane
// branches: an equation's coupling to a neighbour that does not exist is
// exactly zero (and lanes past the last even equation hold identity rows),
// so every lane fetches a clamped, in-range neighbour and adds zero terms.
template <typename TS>
__device__ void pcr_solve(int n, const double* Td, const double* To, const double* rhs, double* x) {
  const int l = threadIdx.x & (kWave - 1);
  const int j0 = 2 * l, j1 = 2 * l + 1;
  const int m = (n + 1) / 2;   // even equations
  const bool v0 = j0 < n, v1 = j1 < n;
  // rows 2l, 2l+1 < 128 lie inside the arrays: read unconditionally, then
  // keep only the rows of the system (rows past n - 1 become identity rows)
  const double tom = To[j0 > 0 ? j0 - 1 : 0], td0 = Td[j0], to0 = To[j0], rh0 = rhs[j0];
  const double td1 = Td[j1], to1 = To[j1], rh1 = rhs[j1];
  const TS a0 = (v0 && j0 > 0) ? (TS)tom : (TS)0;
  const TS b0 = v0 ? (TS)td0 : (TS)1;
  const TS c0 = (v0 && j0 + 1 < n) ? (TS)to0 : (TS)0;
  const TS d0 = v0 ? (TS)rh0 : (TS)0;
  const TS a1 = v1 ? (TS)to0 : (TS)0;
  const TS b1 = v1 ? (TS)td1 : (TS)1;
  const TS c1 = (v1 && j1 + 1 < n) ? (TS)to1 : (TS)0;
  const TS d1 = v1 ? (TS)rh1 : (TS)0;
  const TS r1 = rcp_nr(b1);
  // even equation 2l with odd neighbours 2l-1 (lane l-1; a0 = 0 on lane 0)
  // and 2l+1 (own)
  TS A, Bv, C, Dv;
  {
    const TS orb = lane_prev(r1), oa = lane_prev(a1), oc = lane_prev(c1), od = lane_prev(d1);
    const TS al = -a0 * orb, ga = -c0 * r1;
    A = al * oa;
    C = ga * c1;
    Bv = b0 + al * oc + ga * a1;
    Dv = d0 + al * od + ga * d1;
  }
  if (l >= m) { A = 0; Bv = 1; C = 0; Dv = 0; }
  TS rB = rcp_nr(Bv);
  // one PCR level with the neighbours' (rb, a, c, d) at l - s and l + s;
  // A = 0 when l - s < 0 and C = 0 when l + s >= m: those terms add zero
  auto level = [&](TS rbm, TS am, TS cm, TS dm, TS rbp, TS ap, TS cp, TS dpv) {
    const TS al = -A * rbm, ga = -C * rbp;
    A = al * am;
    C = ga * cp;
    Bv += al * cm;
    Bv += ga * ap;
    Dv += al * dm;
    Dv += ga * dpv;
    rB = rcp_nr(Bv);
  };
  if (1 < m)
    level(lane_prev(rB), lane_prev(A), lane_prev(C), lane_prev(Dv),
          lane_next(rB), lane_next(A), lane_next(C), lane_next(Dv));
  for (int s = 2; s < m; s <<= 1) {
    const int lo = (l >= s ? l - s : l) * 4, hi = (l + s < kWave ? l + s : l) * 4;
    level(lane_get(rB, lo), lane_get(A, lo), lane_get(C, lo), lane_get(Dv, lo),
          lane_get(rB, hi), lane_get(A, hi), lane_get(C, hi), lane_get(Dv, hi));
  }
  const double xe = (double)(Dv * rB);
  // even unknown 2l+2 from lane l+1 (none past the last lane)
  const double xnb = lane_next(xe);
  if (v0) x[j0] = xe;
  if (v1) {
    const TS xn = (j1 + 1 < n) ? (TS)xnb : (TS)0;
    x[j1] = (double)((d1 - a1 * (TS)xe - c1 * xn) * r1);
  }
  wave_sync();
}

// max(a, |b|) in one instruction.  The compiler's fmax first quiets a
// possible signalling NaN in `a` with an extra max; the running maxima here
// only ever hold results of arithmetic, which are never signalling.
__device__ __forceinline__ double max_abs(double a, double b) {
  double r;
  asm("v_max_f64 %0, %1, |%2|" : "=v"(r) : "v"(a), "v"(b));
  return r;
}

// Sum over each aligned group of G lanes (G a power of two <= 64): an
// inclusive DPP scan (row_shr 1/2/4/8 inside rows of 16 lanes, then
// row_bcast 15/31 across rows).  The LAST lane of every group ends holding
// its group's total; other lanes hold partial sums.  Every lane of the
// wavefront must be active.
template <int G>
__device__ __forceinline__ double group_sum(double v) {
  if constexpr (G >= 2) v += dpp_d<0x111, 0xf, true>(v);
  if constexpr (G >= 4) v += dpp_d<0x112, 0xf, true>(v);
  if constexpr (G >= 8) v += dpp_d<0x114, 0xf, true>(v);
  if constexpr (G >= 16) v += dpp_d<0x118, 0xf, true>(v);
  if constexpr (G >= 32) v += dpp_d<0x142, 0xa, false>(v);
  if constexpr (G >= 64) v += dpp_d<0x143, 0xc, false>(v);
  return v;
}

// Row totals (16 lanes) of four values at once.  Two exchange steps
// (partner lane ^ 1, then lane ^ 2) leave every lane with a four-lane
// partial of one value, index ((lane & 1) << 1) | ((lane >> 1) & 1), and two
// rotations of the row by 4 and 8 lanes add its four quads, so every lane
// ends with the row total of its value.
__device__ __forceinline__ double row_sum4(double v0, double v1, double v2, double v3, int lane) {
  const bool b0 = (lane & 1) != 0, b1 = (lane & 2) != 0;
  double ka = b0 ? v2 : v0, kb = b0 ? v3 : v1;
  const double sa = b0 ? v0 : v2, sb = b0 ? v1 : v3;
  ka += dpp_d<0xB1, 0xf, false>(sa);   // quad_perm [1,0,3,2]
  kb += dpp_d<0xB1, 0xf, false>(sb);
  double k = b1 ? kb : ka;
  const double sk = b1 ? ka : kb;
  k += dpp_d<0x4E, 0xf, false>(sk);    // quad_perm [2,3,0,1]
  k += dpp_d<0x124, 0xf, false>(k);    // row_ror:4
  k += dpp_d<0x128, 0xf, false>(k);    // row_ror:8
  return k;
}

// group maximum of non-negative values (same scan, fmax)
template <int G>
__device__ __forceinline__ double group_max(double v) {
  if constexpr (G >= 2) v = fmax(v, dpp_d<0x111, 0xf, true>(v));
  if constexpr (G >= 4) v = fmax(v, dpp_d<0x112, 0xf, true>(v));
  if constexpr (G >= 8) v = fmax(v, dpp_d<0x114, 0xf, true>(v));
  if constexpr (G >= 16) v = fmax(v, dpp_d<0x118, 0xf, true>(v));
  if constexpr (G >= 32) v = fmax(v, dpp_d<0x142, 0xa, false>(v));
  if constexpr (G >= 64) v = fmax(v, dpp_d<0x143, 0xc, false>(v));
  return v;
}

template <int NXM>
struct SlabSh {
  // per-slab sums at the current (or trial) point: Sr[0] = sum u,
  // Sr[1] = sum u^2, Sr[2] = sum g, Sr[3] = sum u g (the Schur quantities
  // sum a, sum a^2, sum a g follow from them, a being affine in u)
  double Sr[4][kMaxNt];
  double W[kMaxNt];      // W_k per slab at the current point
  double rW[kMaxNt];     // 1/W_k
  double lam[kMaxNt];    // multipliers of the slab rows at the current point
  double lamp[kMaxNt];   // lam+ of the pending step
  double Td[kMaxNt], To[kMaxNt], r[kMaxNt], res[kMaxNt], dx[kMaxNt];
  double lamic[NXM], lampic[NXM], ric[NXM], gic[NXM];   // IC rows
  double red[16][4];     // per-wavefront partials: max|g|, p.p, (u-u_hat).p
  double red2[16][2];    // load: max|u_hat|, non-finite; second-order trial: q.q, (u-u_hat).q
  double scal[6];        // IC rows: sum a_0 r_ic, max|h_ic|, sum|h_ic|; [3] second-order
                         // sum a_0 h_ic; [4] dlam_0 of the pending step; [5] max|lam+_ic|
  int flag[5];           // done, accepted, backtrack, line-search outcome, local phase
};

// The kernel's LDS in one object, the large u_hat staging last, so that every
// small array sits below 64 KiB and is reached with immediate offsets.
template <int NXM, int UHN, typename TS>
struct SlabLds {
  SlabSh<NXM> sh;
  double uhl[UHN];   // u_hat (forward) or u* + grad_u (adjoint)
};

template <int NW, int G, int XPL, int RMAX, int UHN, typename TS, bool SOC>
__global__ __launch_bounds__(NW * kWave, 1) void slab_kernel(KernelArgs A) {
  constexpr int NT = NW * kWave;   // threads
  constexpr int NG = NT / G;       // slab groups per round
  constexpr int GPW = kWave / G;   // groups per wavefront
  constexpr int NXM = G * XPL;     // widest grid of the class
  static_assert(NW <= 16 && (NW & (NW - 1)) == 0 && G <= kWave && NG * RMAX <= kMaxNt &&
                NXM % kWave == 0, "slab class");

  const int sid = A.order[blockIdx.x];
  const snap_sample_desc D = A.descs[sid];
  const int nx = D.nx, nt = D.nt, nr = nt - 1;
  const bool f2 = (D.family == SNAP_FISHER_KPP);
  const double c = f2 ? D.dt * D.p0 : 0.0;
  const double a0c = f2 ? -1.0 - c : 0.0, a1c = f2 ? 2.0 * c : 0.0;
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int w = __builtin_amdgcn_readfirstlane(tid / kWave);   // wave-uniform
  const int grp = tid / G, sub = tid & (G - 1);
  const bool glast = sub == G - 1;
  const bool bwd = A.backward != 0;
  const int64_t vo = D.var_off;

  __shared__ SlabLds<NXM, UHN, TS> lds;
  SlabSh<NXM>& sh = lds.sh;
  double* const uhl = lds.uhl;

  const double* aux = A.aux + D.aux_off;
  const double m0 = f2 ? 0.0 : aux[nx];

  // Group g takes slab ((g + r*GPW) mod NG) + NG*r in round r: round 0 is
  // slab g (slab 0, with the IC rows, on wavefront 0), and each later round
  // moves the wavefronts' blocks of slabs by one, so a partial last round
  // lands on another wavefront than the one that carries the IC rows.
  auto slab_of = [&](int g, int r) { return ((g + r * GPW) & (NG - 1)) + NG * r; };
  auto slab = [&](int r) { return slab_of(grp, r); };
  auto xat = [&](int j) { return sub + G * j; };
  // element (round r, j) sits at k*nx + x
  auto eidx = [&](int r, int j) { return slab(r) * nx + sub + G * j; };
  // The Newton loop re-reads u_hat and the IC targets from LDS in every pass;
  // an opaque copy of the lane's indices keeps the compiler from hoisting
  // those loop-invariant reads into registers (which would not fit).
  auto opaque = [](int v) {
    asm volatile("" : "+v"(v));
    return v;
  };
  // wavefront w holds a slab < nt in round r (uniform over the wavefront):
  // its groups take the block of slabs starting at ((w + r) mod NW)*GPW + NG*r
  auto live = [&](int r) { return ((w + r) & (NW - 1)) * GPW + NG * r < nt; };
  auto coef = [&](int k, double uu) { return k < nr ? a0c + a1c * uu : 0.0; };
  auto wslab = [&](int k, double l) { return k < nr ? fmax(1.0 + 2.0 * c * l, kWFloor) : 1.0; };

  double u[RMAX][XPL], pst[RMAX][XPL];

  // ---------------------------------------------------------------- load
  double umax = 0.0;
  bool nonfinite = false;
  // every load is issued before the first use (indices clamped, no branches);
  // the adjoint reads u* into u and grad_u into pst
  // the forward's IC targets of slab 0 (wavefront 0) load with the field
  double gi0[XPL];
  {
    const double* src = bwd ? A.u + vo : A.uhat + vo;
#pragma unroll
    for (int r = 0; r < RMAX; ++r)
#pragma unroll
      for (int j = 0; j < XPL; ++j) {
        const bool ok = slab(r) < nt && xat(j) < nx;
        const int idx = ok ? eidx(r, j) : 0;
        u[r][j] = src[idx];
        pst[r][j] = bwd ? A.grad_u[vo + idx] : 0.0;
      }
#pragma unroll
    for (int j = 0; j < XPL; ++j) gi0[j] = (!bwd && w == 0) ? aux[xat(j) < nx ? xat(j) : 0] : 0.0;
  }
  // Forward start u = u_hat, lam = 0: g = 0 exactly, so a slab's sums are
  // sum u and sum u^2 of the registers just loaded (slots outside the grid
  // hold 0), formed round by round while later rounds' loads are in flight;
  // on slab 0 the IC rows' h_ic, which is also r_ic here.
  auto start_round = [&](int r) {
    const int k = slab(r);
    const bool kv = k < nt;
    double Su = -0.0, Suu = -0.0;
#pragma unroll
    for (int j = 0; j < XPL; ++j) {
      Su += u[r][j];
      Suu = fma(u[r][j], u[r][j], Suu);
    }
    if constexpr (G == 16) {
      const double t = row_sum4(Su, Suu, 0.0, 0.0, lane);
      const int vi = ((lane & 1) << 1) | ((lane >> 1) & 1);
      if ((lane & 12) == 0 && kv) sh.Sr[vi][k] = t;
    } else {
      Su = group_sum<G>(Su); Suu = group_sum<G>(Suu);
      if (glast && kv) { sh.Sr[0][k] = Su; sh.Sr[1][k] = Suu; sh.Sr[2][k] = 0.0; sh.Sr[3][k] = 0.0; }
    }
    if (r == 0 && w == 0) {
      const double a0 = nr > 0 ? a0c : 0.0, a1 = nr > 0 ? a1c : 0.0;
      double sar = -0.0, hmx = 0.0, h1 = -0.0;
#pragma unroll
      for (int j = 0; j < XPL; ++j) {
        const bool okx = grp == 0 && xat(j) < nx;
        const double uu = u[0][j];
        const double hic = uu - gi0[j];
        if (okx) sh.ric[xat(j)] = hic;
        sar += okx ? (a0 + a1 * uu) * hic : 0.0;
        hmx = fmax(hmx, okx ? fabs(hic) : 0.0);
        h1 += okx ? fabs(hic) : 0.0;
      }
      sar = group_sum<G>(sar); h1 = group_sum<G>(h1); hmx = group_max<G>(hmx);
      if (lane == G - 1) { sh.scal[0] = sar; sh.scal[1] = hmx; sh.scal[2] = h1; }
    }
  };
#pragma unroll
  for (int r = 0; r < RMAX; ++r) {
    const int k = slab(r);
#pragma unroll
    for (int j = 0; j < XPL; ++j) {
      const bool ok = k < nt && xat(j) < nx;
      const double uu = ok ? u[r][j] : 0.0;
      const double hh = ok ? uu + pst[r][j] : 0.0;   // u_hat, or u* + grad_u
      u[r][j] = uu;
      pst[r][j] = 0.0;
      // full-width grids also zero the staging slots of slabs past nt (they
      // lie inside the array), which the unguarded trial pass reads
      if (ok || nx == NXM) uhl[eidx(r, j)] = hh;
      umax = fmax(umax, fabs(hh));
      nonfinite |= !finite(hh) || !finite(uu);
    }
    if (!bwd && live(r)) start_round(r);
    __builtin_amdgcn_sched_barrier(0);
  }
  if (!bwd && lane == 0) { sh.red[w][0] = 0.0; sh.red[w][1] = 0.0; sh.red[w][2] = 0.0; }
  for (int x = tid; x < nx; x += NT) {
    sh.gic[x] = aux[x];
    sh.lamic[x] = 0.0;
    sh.lampic[x] = 0.0;
  }
  // the adjoint takes W at lam*, and its right-hand side J W^{-1} grad_u only,
  // so the multipliers entering the stationarity residual are zero
  int floored = 0;   // adjoint: exact W below the floor somewhere
  for (int k = tid; k < kMaxNt; k += NT) {
    const double l = (bwd && k < nr) ? A.lam[D.row_off + nx + k] : 0.0;
    const double wk = wslab(k, l);
    floored |= k < nr && 1.0 + 2.0 * c * l < kWFloor;
    sh.W[k] = wk;
    sh.rW[k] = rcp_nr(wk);
    sh.lam[k] = 0.0;
    sh.lamp[k] = 0.0;
  }
  floored = __syncthreads_or(floored);
  // Slab sums at a point, in one of two forms (the pass kind is a
  // compile-time constant, so each call site gets its own code):
  //   kPoint  the point u with multipliers lamv (slab rows), lamicv (IC rows);
  //   kStep   first the step p at the current point with lam+ (into pst),
  //           with the merit terms p.p and (u - u_hat).p, then the trial
  //           point u + p; the IC rows' lam+ is formed here, by the lanes that
  //           own slab 0 (lam+_ic = lam_ic + W_0 r_ic - a_0 dlam_0, stored
  //           for the line search and its maximum kept for the penalty);
  // Per slab: sum u, sum u^2, sum g, sum u g, and the IC rows'
  // r_ic = h_ic - g/W_0 (W_0 of the multipliers the sums describe).
  // In the local phase (||h||_inf <= 1e-6 at the current point) the full step
  // is always accepted, so its trial point u + p can go to the output right
  // after the step pass: it is the next iterate. `written` records that the
  // output holds the current iterate.
  bool spec = false, written = false;
  double* const uout = A.u + vo;
  auto sums_pass = [&](const double* lamv, const double* lamicv, auto kind) {
    constexpr int M = decltype(kind)::value;
    constexpr bool step = M == kStep;
    const int xs = opaque(sub), gq = opaque(grp);
    double st = 0.0, pp = -0.0, dd = -0.0;
    // W_0 at the point the sums describe: of lam+ at a trial point, else the
    // stored one (the adjoint keeps W of lam* while its multipliers are zero)
    const double rW0 = step ? rcp_nr(wslab(0, nr > 0 ? lamv[0] : 0.0)) : sh.rW[0];
#pragma unroll
    for (int r = 0; r < RMAX; ++r) {
      if (!live(r)) continue;
      const int k = slab_of(gq, r);
      const int eb = k * nx + xs;   // element (k, xs + G*j) at eb + G*j
      const bool kv = k < nt;
      const bool law = k < nr;
      // per-slab constants: a = a0 + a1 u on law slabs (0 on the last slab);
      // the +1 coefficient of row k-1 on slab k, or the IC multiplier on slab 0
      const double a0 = law ? a0c : 0.0, a1 = law ? a1c : 0.0;
      const double lk = law ? lamv[k] : 0.0;
      const double lkm = (k >= 1 && kv) ? lamv[k - 1] : 0.0;
      const bool ic = r == 0 && k == 0;
      // step at the current point: W of the current multipliers
      const double rWc = (kv && step) ? sh.rW[k] : 1.0;
      const double W0 = (ic && step) ? sh.W[0] : 0.0;
      const double dl0 = (ic && step) ? sh.scal[4] : 0.0;
      // With the multipliers fixed, g is affine in u on a slab:
      // g = (u - u_hat) + gam u + bet, gam = a1 lk, bet = a0 lk + (the +1
      // coefficient's multiplier: row k-1's, or the IC row's on slab 0).
      // The accumulators start at -0, which the first add folds away.
      const double gam = a1 * lk, bet = a0 * lk + lkm;
      double Su = -0.0, Suu = -0.0, Sg = -0.0, Sug = -0.0, sar = -0.0, hmx = 0, h1 = -0.0, lpm = 0;
      // one element (round r, j); IC: the slab-0 lanes' IC terms may apply
      auto elem = [&](int j, auto icc) {
        constexpr bool IC = decltype(icc)::value;
        double uu = u[r][j];
        const double uh = uhl[eb + G * j];
        double bx = bet;
        if (IC && ic) {
          double lm;
          if constexpr (step) {
            lm = sh.lamic[xs + G * j] + (W0 * sh.ric[xs + G * j] - (a0 + a1 * uu) * dl0);
            sh.lampic[xs + G * j] = lm;
            lpm = fmax(lpm, fabs(lm));
          } else {
            lm = lamicv[xs + G * j];
          }
          bx = a0 * lk + lm;
        }
        if constexpr (step) {
          // the trial point is u + p with p rounded first (no contraction),
          // the same value the accepted step gives u
#pragma clang fp contract(off)
          const double d = uu - uh;
          const double jt = fma(uu, gam, d) + bx;
          const double p = -jt * rWc;
          pst[r][j] = p;
          pp = fma(p, p, pp);
          dd = fma(d, p, dd);
          uu = uu + 1.0 * p;
        }
        Su += uu;
        Suu = fma(uu, uu, Suu);
        const double g = fma(uu, gam, uu - uh) + bx;
        Sg += g;
        Sug = fma(uu, g, Sug);
        st = max_abs(st, g);
        if (IC && ic) {
          const double a = a0 + a1 * uu;
          const double gi = sh.gic[xs + G * j];
          const double hic = bwd ? 0.0 : uu - gi;
          const double ric = hic - g * rW0;
          sh.ric[xs + G * j] = ric;
          sar += a * ric;
          hmx = fmax(hmx, fabs(hic));
          h1 += fabs(hic);
        }
      };
      // Full-width grid (nx = G*XPL) outside round 0 of wavefront 0: the only
      // slots outside the grid are whole slabs past nt, which hold u = 0, a
      // zero-filled staging row and zero multipliers, so every term they
      // add is exactly zero and the elements need no guard.
      if (step && nx == NXM && !(r == 0 && w == 0)) {
#pragma unroll
        for (int j = 0; j < XPL; ++j) elem(j, PassKind<0>{});
      } else {
#pragma unroll
        for (int j = 0; j < XPL; ++j)
          if (kv && xat(j) < nx) elem(j, PassKind<1>{});
      }
      if constexpr (G == 16) {
        // a group is a row: one transposed reduction, four lanes write
        const double t = row_sum4(Su, Suu, Sg, Sug, lane);
        const int vi = ((lane & 1) << 1) | ((lane >> 1) & 1);
        if ((lane & 12) == 0 && kv) sh.Sr[vi][k] = t;
      } else {
        Su = group_sum<G>(Su); Suu = group_sum<G>(Suu);
        Sg = group_sum<G>(Sg); Sug = group_sum<G>(Sug);
        if (glast && kv) { sh.Sr[0][k] = Su; sh.Sr[1][k] = Suu; sh.Sr[2][k] = Sg; sh.Sr[3][k] = Sug; }
      }
      if (w == 0 && r == 0) {   // group 0 holds slab 0 and the IC rows
        sar = group_sum<G>(sar); h1 = group_sum<G>(h1); hmx = group_max<G>(hmx);
        if constexpr (step) lpm = group_max<G>(lpm);
        if (lane == G - 1) {
          sh.scal[0] = sar; sh.scal[1] = hmx; sh.scal[2] = h1;
          if constexpr (step) sh.scal[5] = lpm;
        }
      }
      // one round at a time: bounds the values in flight
      __builtin_amdgcn_sched_barrier(0);
    }
    st = wave_max(st);
    if (step) { pp = wave_sum(pp); dd = wave_sum(dd); }
    if (lane == 0) { sh.red[w][0] = st; sh.red[w][1] = pp; sh.red[w][2] = dd; }
  };

  {
    const double mx = wave_max(umax);
    const int nf = __any(nonfinite) ? 1 : 0;
    if (lane == 0) { sh.red2[w][0] = mx; sh.red2[w][1] = (double)nf; }
  }
  lds_barrier();
  double uscale = 0.0, nfin = 0.0;
  for (int q = 0; q < NW; ++q) { uscale = fmax(uscale, sh.red2[q][0]); nfin += sh.red2[q][1]; }
  uscale += 1.0;

  // feasibility row k from the slab sums S1, S2
  auto row_h = [&](int k) -> double {
    return f2 ? sh.Sr[0][k + 1] - sh.Sr[0][k] - c * (sh.Sr[0][k] - sh.Sr[1][k]) : sh.Sr[0][k + 1] - m0;
  };
  // sum of |h| over all rows (IC rows from scal[2]); wavefront 0 only
  auto h1_rows = [&]() -> double {
    double h1 = (lane == 0) ? sh.scal[2] : 0.0;
    for (int k = lane; k < nr; k += kWave) h1 += fabs(row_h(k));
    return wave_sum(h1);
  };

  double mu = 0.0, hinf = 0.0, stinf = 0.0, h1cur = 0.0;
  double lmrow = 0.0;   // max |lam+| over the slab rows of the pending step (wavefront 0)
  int iters = 0, backtracks = 0, refines = 0, status = SNAP_ST_MAX_ITER;
  if (nfin > 0.0) status = SNAP_ST_NONFINITE;
  const int max_it = bwd ? 1 : A.opt.max_newton;
  bool pend = false;   // the sums describe the trial point u + p of a pending step

  if (bwd && status != SNAP_ST_NONFINITE) {
    sums_pass(sh.lam, sh.lamic, PassKind<kPoint>{});
    lds_barrier();
  }

  for (int it = 0; status != SNAP_ST_NONFINITE; ++it) {
    // ------------------------------------------------ wavefront 0: accept, test, solve
    if (w == 0) {
      int done = 0, acc = 0, bt = 0, soc = 0;
      // per-wavefront partials of the last pass, lane q holding wavefront q's
      const int qi = lane < NW ? lane : 0;
      const bool qv = lane < NW;
      const double qst = sh.red[qi][0], qpp = sh.red[qi][1], qdd = sh.red[qi][2];
      // a pending step's multipliers and its IC rows' max |lam+| are read with
      // the sums, so an accepted step needs no further LDS round trip
      const double sc5 = sh.scal[5];
      static_assert(kMaxNt == 2 * kWave, "two rows per lane");
      const double lp0 = sh.lamp[lane], lp1 = sh.lamp[lane + kWave];
      double lpic[NXM / kWave];
#pragma unroll
      for (int e = 0; e < NXM / kWave; ++e) lpic[e] = sh.lampic[lane + kWave * e];
      // rows k = lane and lane + 64 (nr <= 127): h from the slab sums, once
      double hk[2];
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const int k = lane + kWave * e;
        // reads unconditional (k + 1 clamped into the array), value kept for rows < nr
        const int k1 = k + 1 < kMaxNt ? k + 1 : k;
        const double s1k = sh.Sr[0][k], s1n = sh.Sr[0][k1], s2k = s1k - sh.Sr[1][k];
        const double h = f2 ? s1n - s1k - c * s2k : s1n - m0;
        hk[e] = (k < nr && !bwd) ? h : 0.0;
      }
      double h1 = (lane == 0) ? sh.scal[2] : 0.0;
      h1 += fabs(hk[0]) + fabs(hk[1]);
      // the three reductions are independent (the merit terms are formed even
      // when no step is pending; they are then unused)
      h1 = wave_sum(h1);
      const double pp = wave_sum(qv ? qpp : 0.0), dd = wave_sum(qv ? qdd : 0.0);
      if (pend) {
        // penalty mu >= 1.1 ||lam+||_inf of the pending step (IC rows' part
        // from the trial pass)
        mu = bcast_first(fmax(mu, 1.1 * fmax(lmrow, sc5) + 1e-8));
        // Armijo test of phi = 1/2||u - u_hat||^2 + mu||h||_1 at alpha = 1; the
        // change is formed from differences, d.p + p.p/2 + mu(||h_t||_1 - ||h||_1),
        // so rounding of the large sums in phi never decides.  Local phase
        // (||h||_inf <= 1e-6): full Newton steps.
        const double dphi = dd - mu * h1cur;
        const double dphit = dd + 0.5 * pp + mu * (h1 - h1cur);
        // (with W >= 0.1 the step is a descent direction of the merit unless
        // it is zero; a zero step is taken, any other must pass the test)
        acc = (dphit <= 1e-4 * dphi) || !(pp > 0.0) || hinf <= 1e-6;
        // rejected: a second-order correction is tried only when the full step
        // increased the constraint violation (the curvature of h is what failed)
        soc = SOC && !acc && h1 > h1cur;
        if (acc) {
          // (u += p is applied by every wavefront after the barrier).  Rows
          // past nr hold lam+ = 0 and W = 1 throughout, so all 128 entries
          // are rewritten without a branch.
#pragma unroll
          for (int e = 0; e < 2; ++e) {
            const int k = lane + kWave * e;
            const double l = e ? lp1 : lp0;
            const double wk = wslab(k, l);
            sh.lam[k] = l;
            sh.W[k] = wk;
            sh.rW[k] = rcp_nr(wk);
          }
#pragma unroll
          for (int e = 0; e < NXM / kWave; ++e) sh.lamic[lane + kWave * e] = lpic[e];
          wave_sync();
        } else {
          bt = 1;
        }
      }
      if (!bt) {
        double hmax = (lane == 0) ? sh.scal[1] : 0.0;
        bool nf = false;
        // rows k = lane, lane + 64: every read issued up front (index k + 1
        // clamped into the arrays); entries past nr - 1 are written too and
        // never read (the solve reads rows < nr only)
        const double sar0 = sh.scal[0];
        double rWk[2], rWk1[2], sad[2], sdn[2], sa2[2], san[2];
        // an opaque row index: these reads are issued again here rather than
        // kept live in registers from the test above
        const int lo = opaque(lane);
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          const int k = lo + kWave * e;
          const int k1 = k + 1 < kMaxNt ? k + 1 : k;
          rWk[e] = sh.rW[k]; rWk1[e] = sh.rW[k1];
          // sum a g, sum a^2 on slab k and sum a on slab k + 1 from the raw sums
          // (a = a0 + a1 u on slabs < nr, 0 on the last)
          const double su = sh.Sr[0][k], suu = sh.Sr[1][k], sg = sh.Sr[2][k], sug = sh.Sr[3][k];
          const double su1 = sh.Sr[0][k1], sg1 = sh.Sr[2][k1];
          const double ak0 = k < nr ? a0c : 0.0, ak1 = k < nr ? a1c : 0.0;
          const double an0 = k1 < nr ? a0c : 0.0, an1 = k1 < nr ? a1c : 0.0;
          const double cnt = (double)nx;
          sad[e] = ak0 * sg + ak1 * sug;
          sdn[e] = sg1;
          sa2[e] = ak0 * ak0 * cnt + 2.0 * ak0 * ak1 * su + ak1 * ak1 * suu;
          san[e] = an0 * cnt + an1 * su1;
        }
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          const int k = lane + kWave * e;
          double rk = hk[e] - (sad[e] * rWk[e] + sdn[e] * rWk1[e]);
          if (k == 0) rk -= sar0;
          sh.r[k] = rk;
          sh.Td[k] = (k == 0 ? 0.0 : sa2[e] * rWk[e]) + (double)nx * rWk1[e];
          sh.To[k] = (k + 1 < nr) ? san[e] * rWk1[e] : 0.0;
          hmax = fmax(hmax, fabs(hk[e]));   // hk = 0 past nr - 1
          nf |= !finite(hk[e]);
        }
        hmax = wave_max(hmax);
        nf = __any(nf);
        const double stmax = wave_max(qv ? qst : 0.0);
        if (!bwd) {
          hinf = bcast_first(hmax); stinf = bcast_first(stmax); h1cur = bcast_first(h1);
          if (nf || !finite(hmax) || !finite(stmax)) done = 2;
          else if (hmax <= A.opt.tol_h && stmax <= A.opt.tol_s * uscale) done = 1;
          else if (it >= max_it) done = 3;
        }
        wave_sync();
        if (!done && nr > 0) {
          pcr_solve<TS>(nr, sh.Td, sh.To, sh.r, sh.lamp);
          if constexpr (sizeof(TS) != sizeof(double)) {
            // float32 solve, float64 residual and refinement
            constexpr int max_ref = 4;
            // rows k = lane, lane + 64; reads unconditional with clamped
            // neighbours, values kept for rows < nr
            double rn = 0.0;
#pragma unroll
            for (int e = 0; e < 2; ++e) {
              const int k = lane + kWave * e;
              const double rk = sh.r[k];
              rn = fmax(rn, k < nr ? fabs(rk) : 0.0);
            }
            rn = wave_max(rn);
            for (int ref = 0; ref < max_ref; ++ref) {
              double resmax = 0.0;
#pragma unroll
              for (int e = 0; e < 2; ++e) {
                const int k = lane + kWave * e;
                const int km = k > 0 ? k - 1 : 0, kp = k + 1 < kMaxNt ? k + 1 : k;
                const double tdk = sh.Td[k], lk = sh.lamp[k], tom = sh.To[km], lkm = sh.lamp[km];
                const double tok = sh.To[k], lkp = sh.lamp[kp], rk = sh.r[k];
                double tx = tdk * lk;
                tx += k > 0 ? tom * lkm : 0.0;
                tx += k + 1 < nr ? tok * lkp : 0.0;
                const double res = rk - tx;
                if (k < nr) sh.res[k] = res;
                resmax = fmax(resmax, k < nr ? fabs(res) : 0.0);
              }
              resmax = wave_max(resmax);
              wave_sync();
              // a Newton step only needs its residual well below the feasibility
              // tolerance, and far from the solution (||h||_inf > 1e-6) only a
              // good descent direction; the adjoint is solved to working precision
              const double target = bwd ? 1e-15 * rn
                                        : (hinf > 1e-6 ? 1e-6 * rn : fmax(1e-15 * rn, 0.1 * A.opt.tol_h));
              if (!(resmax > target)) break;
              pcr_solve<TS>(nr, sh.Td, sh.To, sh.res, sh.dx);
#pragma unroll
              for (int e = 0; e < 2; ++e) {
                const int k = lane + kWave * e;
                const double lk = sh.lamp[k], dxk = sh.dx[k];
                if (k < nr) sh.lamp[k] = lk + dxk;
              }
              wave_sync();
              ++refines;
            }
          }
        }
        if (!done) {
          // sh.lamp holds dlam: keep dlam_0 for the IC rows' multipliers (formed
          // from the eliminated block by the next pass), then lam+ = lam + dlam
          const double l0 = nr > 0 ? sh.lamp[0] : 0.0;
          if (lane == 0) sh.scal[4] = l0;
          double lm = 0.0;
#pragma unroll
          for (int e = 0; e < 2; ++e) {
            const int k = lane + kWave * e;
            // rows past nr - 1 hold zeros in both (no branch needed)
            const double l = sh.lamp[k] + sh.lam[k];
            sh.lamp[k] = l;
            lm = fmax(lm, fabs(l));
          }
          lmrow = bcast_first(wave_max(lm));
        }
      }
      if (lane == 0) {
        sh.flag[0] = done; sh.flag[1] = acc; sh.flag[2] = bt | (soc << 1);
        sh.flag[4] = !bwd && !bt && hinf <= 1e-6;   // the coming step will be accepted
      }
    }
    lds_barrier();
    const int done = sh.flag[0], acc = sh.flag[1], bt = sh.flag[2] & 1, soc_try = sh.flag[2] >> 1;
    spec = sh.flag[4] != 0;
    if (acc) {
#pragma unroll
      for (int r = 0; r < RMAX; ++r)
#pragma unroll
        for (int j = 0; j < XPL; ++j) u[r][j] += 1.0 * pst[r][j];
      ++iters;
    }
    if (bt) {
      ++backtracks;   // the full step was rejected
      // ---------------------------------------------- second-order correction
      // One try before halving: with the Schur system still assembled at u
      // (the factor is reused), solve S z = h(u + p) and move to
      // u + q, q = p + p_soc, p_soc = -W^{-1} J(u)^T z; the same Armijo test
      // (directional derivative of p) decides.
      if (SOC && soc_try) {
        if (w == 0) {
          // IC rows at u + p (group 0); with the IC block eliminated the
          // reduced right-hand side is h_k(u+p), minus sum_x a_0(x) h_ic(x) on row 0
          double sar = 0.0;
          if (grp == 0) {
#pragma unroll
            for (int j = 0; j < XPL; ++j) {
              const int x = xat(j);
              if (x < nx) {
                const double hic = (u[0][j] + 1.0 * pst[0][j]) - sh.gic[x];
                sh.ric[x] = hic;
                sar += coef(0, u[0][j]) * hic;
              }
            }
          }
          sar = group_sum<G>(sar);
          if (lane == G - 1) sh.scal[3] = sar;
          wave_sync();
          for (int k = lane; k < nr; k += kWave) sh.res[k] = row_h(k) - (k == 0 ? sh.scal[3] : 0.0);
          wave_sync();
          if (nr > 0) pcr_solve<TS>(nr, sh.Td, sh.To, sh.res, sh.dx);
          const double z0 = nr > 0 ? sh.dx[0] : 0.0;
          const double W0 = sh.W[0];
          if (grp == 0) {
#pragma unroll
            for (int j = 0; j < XPL; ++j) {
              const int x = xat(j);
              if (x < nx) sh.ric[x] = W0 * sh.ric[x] - coef(0, u[0][j]) * z0;   // z_ic
            }
          }
        }
        lds_barrier();
        // trial u + q: slab sums for h, the IC rows, and the merit terms of q
        {
          const int xs = opaque(sub), gq = opaque(grp);
          double qq = 0.0, dq = 0.0;
#pragma unroll
          for (int r = 0; r < RMAX; ++r) {
            if (!live(r)) continue;
            const int k = slab_of(gq, r);
            const int eb = k * nx + xs;
            const bool kv = k < nt;
            const double zk = (k < nr) ? sh.dx[k] : 0.0;
            const double zkm = (k >= 1 && kv) ? sh.dx[k - 1] : 0.0;
            const double rW = kv ? sh.rW[k] : 1.0;
            double Su = 0, Suu = 0, h1 = 0;
#pragma unroll
            for (int j = 0; j < XPL; ++j) {
              const int x = xat(j);
              if (kv && x < nx) {
                const double uu = u[r][j];
                const double zm = (r == 0 && k == 0) ? sh.ric[xs + G * j] : zkm;
                const double q = pst[r][j] - (coef(k, uu) * zk + zm) * rW;
                const double us = uu + q;
                const double d = uu - uhl[eb + G * j];
                qq += q * q;
                dq += d * q;
                Su += us; Suu += us * us;
                if (r == 0 && k == 0) h1 += fabs(us - sh.gic[xs + G * j]);
              }
            }
            Su = group_sum<G>(Su); Suu = group_sum<G>(Suu);
            if (glast && kv) { sh.Sr[0][k] = Su; sh.Sr[1][k] = Suu; }
            if (w == 0 && r == 0) {
              h1 = group_sum<G>(h1);
              if (lane == G - 1) sh.scal[2] = h1;
            }
          }
          qq = wave_sum(qq); dq = wave_sum(dq);
          if (lane == 0) { sh.red2[w][0] = qq; sh.red2[w][1] = dq; }
        }
        lds_barrier();
        if (w == 0) {
          double dd = 0.0, qq = 0.0, dq = 0.0;
          for (int q = 0; q < NW; ++q) { dd += sh.red[q][2]; qq += sh.red2[q][0]; dq += sh.red2[q][1]; }
          const double dphi = dd - mu * h1cur;
          const double dphis = dq + 0.5 * qq + mu * (h1_rows() - h1cur);
          const int good = (dphis <= 1e-4 * dphi) ? 1 : 0;
          if (lane == 0) sh.flag[3] = good;
        }
        lds_barrier();
        if (sh.flag[3]) {
          // accept u + q with lam+ (the multipliers of the full step)
          const int xs = opaque(sub), gq = opaque(grp);
#pragma unroll
          for (int r = 0; r < RMAX; ++r) {
            const int k = slab_of(gq, r);
            const bool kv = k < nt;
            const double zk = (k < nr) ? sh.dx[k] : 0.0;
            const double zkm = (k >= 1 && kv) ? sh.dx[k - 1] : 0.0;
            const double rW = kv ? sh.rW[k] : 1.0;
#pragma unroll
            for (int j = 0; j < XPL; ++j) {
              const int x = xat(j);
              if (kv && x < nx) {
                const double uu = u[r][j];
                const double zm = (r == 0 && k == 0) ? sh.ric[xs + G * j] : zkm;
                u[r][j] = uu + (pst[r][j] - (coef(k, uu) * zk + zm) * rW);
              }
            }
          }
          lds_barrier();   // every lane has read z and the IC correction
          for (int k = tid; k < nr; k += NT) {
            const double l = sh.lamp[k];
            const double wk = wslab(k, l);
            sh.lam[k] = l;
            sh.W[k] = wk;
            sh.rW[k] = rcp_nr(wk);
          }
          for (int x = tid; x < nx; x += NT) sh.lamic[x] = sh.lampic[x];
          ++iters;
          lds_barrier();
          sums_pass(sh.lam, sh.lamic, PassKind<kPoint>{});
          lds_barrier();
          pend = false;
          continue;
        }
        ++backtracks;   // the corrected step was rejected too
      }
      // ---------------------------------------------- backtracking (alpha < 1)
      double alpha = 1.0;
      int ok = 0;
      for (int ls = 1; ls <= A.opt.max_ls; ++ls) {
        alpha *= 0.5;
        const int xs = opaque(sub), gq = opaque(grp);
#pragma unroll
        for (int r = 0; r < RMAX; ++r) {
          if (!live(r)) continue;
          const int k = slab_of(gq, r);
          double Su = 0, Suu = 0, h1 = 0;
#pragma unroll
          for (int j = 0; j < XPL; ++j) {
            const int x = xat(j);
            if (k < nt && x < nx) {
              const double ut = u[r][j] + alpha * pst[r][j];
              Su += ut; Suu += ut * ut;
              if (r == 0 && k == 0) h1 += fabs(ut - sh.gic[xs + G * j]);
            }
          }
          Su = group_sum<G>(Su); Suu = group_sum<G>(Suu);
          if (glast && k < nt) { sh.Sr[0][k] = Su; sh.Sr[1][k] = Suu; }
          if (w == 0 && r == 0) {
            h1 = group_sum<G>(h1);
            if (lane == G - 1) sh.scal[2] = h1;
          }
        }
        lds_barrier();
        if (w == 0) {
          double pp = 0.0, dd = 0.0;
          for (int q = 0; q < NW; ++q) { pp += sh.red[q][1]; dd += sh.red[q][2]; }
          const double dphi = dd - mu * h1cur;
          const double dphit = alpha * dd + 0.5 * alpha * alpha * pp + mu * (h1_rows() - h1cur);
          const int good = (dphit <= 1e-4 * alpha * dphi) || !(pp > 0.0) ? 1 : 0;
          if (lane == 0) sh.flag[3] = good;
        }
        lds_barrier();
        if (sh.flag[3]) { ok = 1; break; }
        ++backtracks;
      }
      if (!ok) {
        status = SNAP_ST_LS_FAIL;
        break;
      }
      // accept: u += alpha p, lam += alpha (lam+ - lam); fresh sums at the new point
#pragma unroll
      for (int r = 0; r < RMAX; ++r)
#pragma unroll
        for (int j = 0; j < XPL; ++j) u[r][j] += alpha * pst[r][j];
      for (int k = tid; k < nr; k += NT) {
        const double l = sh.lam[k] + alpha * (sh.lamp[k] - sh.lam[k]);
        const double wk = wslab(k, l);
        sh.lam[k] = l;
        sh.W[k] = wk;
        sh.rW[k] = rcp_nr(wk);
      }
      for (int x = tid; x < nx; x += NT) sh.lamic[x] += alpha * (sh.lampic[x] - sh.lamic[x]);
      ++iters;
      lds_barrier();
      sums_pass(sh.lam, sh.lamic, PassKind<kPoint>{});
      lds_barrier();
      pend = false;
      continue;
    }
    if (done) {
      status = done == 1 ? SNAP_ST_CONVERGED : (done == 2 ? SNAP_ST_NONFINITE : SNAP_ST_MAX_ITER);
      break;
    }
    if (bwd) {
      // the adjoint is the step of the linearized system: write it and stop
      const int xs = opaque(sub), gq = opaque(grp);
#pragma unroll
      for (int r = 0; r < RMAX; ++r) {
        if (!live(r)) continue;
        const int k = slab_of(gq, r);
        const double lk = (k < nr) ? sh.lamp[k] : 0.0;
        const double lkm = (k >= 1 && k < nt) ? sh.lamp[k - 1] : 0.0;
        const double rW = k < nt ? sh.rW[k] : 1.0;
#pragma unroll
        for (int j = 0; j < XPL; ++j) {
          const int x = xat(j);
          if (k < nt && x < nx) {
            const double uu = u[r][j];
            // IC rows: lam_ic = 0, so the increment is W_0 r_ic - a_0 dlam_0
            const double lic = (r == 0 && k == 0) ? sh.W[0] * sh.ric[x] - coef(0, uu) * sh.scal[4] : 0.0;
            const int e = k * nx + xs + G * j;
            const double jt = (uu - uhl[e]) + coef(k, uu) * lk + lkm + lic;
            A.grad_uhat[vo + e] = -jt * rW;
          }
        }
      }
      status = floored ? SNAP_ST_HESSIAN_FLOOR : SNAP_ST_CONVERGED;
      break;
    }
    // ------------------------------------------------ step and trial point at alpha = 1
    written = spec;
    sums_pass(sh.lamp, sh.lampic, PassKind<kStep>{});
    if (spec) {
      // the coming acceptance gives u + p: write it now (the same operation
      // as the update below), the stores drain while wavefront 0 tests
      const int xs = opaque(sub), gq = opaque(grp);
#pragma unroll
      for (int r = 0; r < RMAX; ++r) {
        const int k = slab_of(gq, r);
#pragma unroll
        for (int j = 0; j < XPL; ++j) {
          const int x = xat(j);
          if (k < nt && x < nx) uout[k * nx + xs + G * j] = u[r][j] + 1.0 * pst[r][j];
        }
      }
    }
    lds_barrier();
    pend = true;
  }

  // ---------------------------------------------------------------- outputs
  if (!bwd) {
    // (the field is already in place when the last step pass wrote its trial
    // point and that step was accepted, which the local phase guarantees)
    const int xs = opaque(sub), gq = opaque(grp);
    if (!written) {
#pragma unroll
      for (int r = 0; r < RMAX; ++r) {
        const int k = slab_of(gq, r);
#pragma unroll
        for (int j = 0; j < XPL; ++j) {
          const int x = xat(j);
          if (k < nt && x < nx) A.u[vo + k * nx + xs + G * j] = u[r][j];
        }
      }
    }
    for (int x = tid; x < nx; x += NT) A.lam[D.row_off + x] = sh.lamic[x];
    for (int k = tid; k < nr; k += NT) A.lam[D.row_off + nx + k] = sh.lam[k];
  }
  if (tid == 0) {
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

// ------------------------------------------------------------------ classes
// (waves, lanes per slab group, x per lane, rounds, u_hat LDS capacity)
struct SlabCfg { int nw, g, xpl, rmax, uhn; };
constexpr SlabCfg kCfg[] = {
    {8, 16, 4, 1, 2048},     // 0: nx <= 64,  nt <= 32
    {8, 8, 8, 2, 8192},      // 1: nx <= 64,  nt <= 128
    {8, 16, 8, 4, 16384},    // 2: nx <= 128, nt <= 128
};
constexpr int kNumCfg = sizeof(kCfg) / sizeof(kCfg[0]);
constexpr int kWideBase = 100;   // classes >= 100: the wide-grid kernel

bool cfg_fits(const SlabCfg& f, int nx, int nt) {
  return nx >= 1 && nt >= 1 && nx <= f.g * f.xpl && nt <= kMaxNt &&
         nt <= (f.nw * kWave / f.g) * f.rmax && nx * nt <= f.uhn;
}

// the second-order-correction try (SNAP_FLAG_SOC) is built into its own
// instantiation, so the default kernel carries none of its registers
template <int I, typename TS>
void launch_cfg(const KernelArgs& a, hipStream_t st) {
  constexpr SlabCfg f = kCfg[I];
  if (a.opt.flags & SNAP_FLAG_SOC)
    hipLaunchKernelGGL((slab_kernel<f.nw, f.g, f.xpl, f.rmax, f.uhn, TS, true>), dim3(a.count),
                       dim3(f.nw * kWave), 0, st, a);
  else
    hipLaunchKernelGGL((slab_kernel<f.nw, f.g, f.xpl, f.rmax, f.uhn, TS, false>), dim3(a.count),
                       dim3(f.nw * kWave), 0, st, a);
}

template <typename TS>
int launch_index(const KernelArgs& a, int i, hipStream_t st) {
  switch (i) {
    case 0: launch_cfg<0, TS>(a, st); break;
    case 1: launch_cfg<1, TS>(a, st); break;
    case 2: launch_cfg<2, TS>(a, st); break;
    default: return SNAP_EUNSUPPORTED;
  }
  return 0;
}

}  // namespace

// Kernel class of an (nx, nt) shape: the first class whose grid capacity and
// u_hat staging cover it; wider grids go to the wide-grid kernel.
int slab_class(int nx, int nt) {
  for (int i = 0; i < kNumCfg; ++i)
    if (cfg_fits(kCfg[i], nx, nt)) return i;
  const int wc = slab_wide_class(nx, nt);
  return wc < 0 ? -1 : kWideBase + wc;
}

// Classes the autotuner may choose between for a shape: every grouped class
// whose capacity covers it (the default first), or the wide-grid class.
int slab_variants(int nx, int nt, int* out, int cap) {
  int n = 0;
  const int d = slab_class(nx, nt);
  if (d < 0 || cap < 1) return 0;
  out[n++] = d;
  if (d >= kWideBase) return n;
  for (int i = 0; i < kNumCfg && n < cap; ++i)
    if (i != d && cfg_fits(kCfg[i], nx, nt)) out[n++] = i;
  return n;
}

// wavefronts per workgroup of a class (for plan descriptions)
int slab_waves(int cls) { return cls >= kWideBase ? 8 : (cls >= 0 && cls < kNumCfg ? kCfg[cls].nw : 0); }

// Host entry used by the plan: one workgroup per listed sample; every sample
// of the launch belongs to kernel class `cls` (shapes may differ).
int slab_launch(const KernelArgs& a, int cls, bool mixed, hipStream_t st) {
  if (a.count == 0) return 0;
  if (cls >= kWideBase) return slab_wide_launch(a, cls - kWideBase, mixed, st);
  const int rc = mixed ? launch_index<float>(a, cls, st) : launch_index<double>(a, cls, st);
  if (rc) return rc;
  return hipGetLastError() == hipSuccess ? 0 : SNAP_EHIP;
}

}  // namespace snap
