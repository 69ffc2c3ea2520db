// Device-side building blocks of the CPR kernels: compact tables, Euler
// fluxes, the Rusanov face flux and the one-dimensional line operations
// every sweep applies (extrapolation to both faces, flux evaluation,
// derivative of the flux interpolant).
//
// The forward kernels are compiled without floating-point contraction and
// spell every fused multiply-add out (r_fma), so each expression rounds
// exactly as written and the x and y sweeps, which run the same code on
// transposed data, round identically.
#pragma once

#include <hip/hip_runtime.h>

#include "cpr_internal.h"

namespace cpr {

// Tables for N1 = P+1 points in the compute type R (kernel argument). Both
// point sets (Gauss and Gauss-Lobatto) are symmetric about the element
// centre, so the tables are too: D[N1-1-i][N1-1-l] = -D[i][l], l_l(+1) = l_{N1-1-l}(-1) and
// gR'(xi_i) = -gL'(xi_{N1-1-i}); the host tables hold these identities
// exactly. Only the independent half is passed (rows i <= N1/2 of D, with
// the centre row's own symmetry, l(-1) and gL'), which halves the scalar
// registers the tables occupy; the accessors rebuild every entry by an
// exact negation or index mirror.
template <typename R, int N1>
struct KTab {
  static constexpr int H = (N1 + 1) / 2;  // rows kept; row H-1 is the centre row for odd N1
  R Dh[H][N1];
  R em_[N1];
  R gL_[N1];
  R gam, gm1;  // gamma and gamma - 1
  R rdx, rdy;  // -2/dx and -2/dy: the reference-to-physical derivative factors
  __device__ __forceinline__ R D(int i, int l) const {
    if (i < N1 - 1 - i) return Dh[i][l];
    if (i > N1 - 1 - i) return -Dh[N1 - 1 - i][N1 - 1 - l];
    // centre row of an odd rule: antisymmetric about the centre, zero there
    if (l < N1 - 1 - l) return Dh[i][l];
    if (l > N1 - 1 - l) return -Dh[i][N1 - 1 - l];
    return R(0);
  }
  __device__ __forceinline__ R em(int l) const { return em_[l]; }
  __device__ __forceinline__ R ep(int l) const { return em_[N1 - 1 - l]; }
  __device__ __forceinline__ R gL(int i) const { return gL_[i]; }
  __device__ __forceinline__ R gR(int i) const { return -gL_[N1 - 1 - i]; }
};

template <typename R, int N1>
inline KTab<R, N1> make_ktab(const Tables1D& T, const Geometry& G) {
  KTab<R, N1> k;
  k.gam = (R)G.gamma;
  k.gm1 = (R)(G.gamma - 1.0);
  k.rdx = (R)(-2.0 / G.dx);
  k.rdy = (R)(-2.0 / G.dy);
  for (int i = 0; i < KTab<R, N1>::H; ++i)
    for (int l = 0; l < N1; ++l) k.Dh[i][l] = (R)T.D[i][l];
  for (int i = 0; i < N1; ++i) {
    k.em_[i] = (R)T.em[i];
    k.gL_[i] = (R)T.gLp[i];
  }
  return k;
}

template <typename R>
__device__ __forceinline__ R r_fma(R a, R b, R c) {
  return fma(a, b, c);
}

// 1/x: the hardware reciprocal estimate refined by Newton's iteration
// r <- r + r (1 - x r), which doubles the number of correct bits per step;
// two steps take the float64 estimate to full precision (about 1 ulp). The
// float32 estimate is already accurate to 1 ulp.
__device__ __forceinline__ double recip(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}
__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }

// sqrt(x) for positive, normal x: the hardware estimate y of 1/sqrt(x)
// refined by the coupled Newton iteration for s = x y -> sqrt(x) and
// h = y/2 -> 1/(2 sqrt(x)) (Markstein's method), then one correction with
// the residual x - s^2. It skips the rescaling of tiny and huge arguments
// that the library square root carries; the sound speeds here never need it
// (a state with p <= 0 or rho <= 0 is flagged as non-physical).
__device__ __forceinline__ double sqrt_pos(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  double s = x * y, h = 0.5 * y;
  const double r = fma(-s, h, 0.5);
  s = fma(s, r, s);
  h = fma(h, r, h);
  const double d = fma(-s, s, x);
  return fma(d, h, s);
}
__device__ __forceinline__ float sqrt_pos(float x) { return sqrtf(x); }

// a*b + c*d rounded as two products and one sum, never fused: the result is
// the same when the two pairs are swapped, which keeps every kernel's
// rounding invariant under the x <-> y transposition of the data.
__device__ __forceinline__ double sym_dot2(double a, double b, double c, double d) {
  return __dadd_rn(__dmul_rn(a, b), __dmul_rn(c, d));
}
__device__ __forceinline__ float sym_dot2(float a, float b, float c, float d) {
  return __fadd_rn(__fmul_rn(a, b), __fmul_rn(c, d));
}

__device__ __forceinline__ double sym_add(double a, double b) { return __dadd_rn(a, b); }
__device__ __forceinline__ float sym_add(float a, float b) { return __fadd_rn(a, b); }

// Fixed-order dot product used for every face extrapolation, so that the two
// elements sharing a face compute bit-identical face states.
template <int N1, typename R, typename C>
__device__ __forceinline__ R dot_n(C c, const R* v) {
  R s = c(0) * v[0];
#pragma unroll
  for (int n = 1; n < N1; ++n) s = r_fma(c(n), v[n], s);
  return s;
}

// Flux of the Euler equations in direction AX (0: f, 1: g) at state q;
// also returns the normal velocity, the pressure and 1/rho.
template <int AX, typename R>
__device__ __forceinline__ void euler_flux(const R q[4], R gm1, R F[4], R& un, R& p, R& ir) {
  ir = recip(q[0]);
  un = q[1 + AX] * ir;
  p = gm1 * r_fma(-(R(0.5) * sym_dot2(q[1], q[1], q[2], q[2])), ir, q[3]);
  F[0] = q[1 + AX];
  F[1] = q[1] * un;
  F[2] = q[2] * un;
  F[1 + AX] = r_fma(q[1 + AX], un, p);
  F[3] = un * (q[3] + p);
}

template <typename R>
__device__ __forceinline__ bool nonphysical(R rho, R p) {
  return !(rho > R(0)) || !(p > R(0));
}

// Rusanov flux across a face with normal +x (AX=0) or +y (AX=1):
// 1/2 (F(qL) + F(qR)) - 1/2 lam (qR - qL), lam = max(|u_n| + c).
template <int AX, typename R>
__device__ __forceinline__ void rusanov(const R qL[4], const R qR[4], R gam, R gm1, R Fh[4],
                                        bool& bad) {
  R fL[4], fR[4], unL, pL, irL, unR, pR, irR;
  euler_flux<AX>(qL, gm1, fL, unL, pL, irL);
  euler_flux<AX>(qR, gm1, fR, unR, pR, irR);
  const R lL = fabs(unL) + sqrt_pos(gam * pL * irL);
  const R lR = fabs(unR) + sqrt_pos(gam * pR * irR);
  const R lam = (lL >= lR) ? lL : lR;
#pragma unroll
  for (int k = 0; k < 4; ++k) Fh[k] = r_fma(-(R(0.5) * lam), qR[k] - qL[k], R(0.5) * (fL[k] + fR[k]));
  bad = bad || nonphysical(qL[0], pL) || nonphysical(qR[0], pR);
}

// ---- Deviation form of the float32 residual ----
// The float32 (FP32-bulk) residual rounds deviations from a reference state
// instead of full flux values. Each element line takes its first solution
// point q_r (float64) as reference; the line works with d = q - q_r, formed
// in float64 and then rounded. The rows of D sum to zero and the
// extrapolation rows to one, so D F = D (F - F(q_r)), and every face term
// F_face - f_face is a difference of deviations once the Rusanov flux is
// written in the same frame; F(q_r) itself is never formed. A neighbour's
// face state enters a line's frame as its own-frame value plus the
// difference of the two references (float64, then rounded). The flux
// deviation dF = F(q_r + d) - F(q_r) is written with the product rule from
// d and the reference's primitive values, so its rounding scales with d:
//   du_n = (dm_n - u_n,r drho) / rho,
//   dK = ((m_r + dm/2) . dm - K_r drho) / rho      (K = |m|^2 / (2 rho)),
//   dp = (g-1)(dE - dK),
//   dF = (dm_n, m_n,r du_n + dm_n u_n + dp, m_t,r du_n + dm_t u_n,
//         du_n (E_r + p_r + dE + dp) + u_n,r (dE + dp)).
// Everything is written in line-normal (n) and line-tangential (t) terms, so
// the x and y sweeps round transposed data identically.
template <typename R>
struct DevRef {
  R rho, mn, mt, un, ut, p, H, K;  // H = E + p, K = rho |V|^2 / 2 of the reference
};

// Reference constants for a line along AX from its reference state: the
// float64 values rounded, and the primitive values formed from those in R.
// Any consistent constants serve: F(q_r) itself never enters, and an error
// in a constant only scales terms that are products with a deviation.
template <int AX, typename R>
__device__ __forceinline__ DevRef<R> dev_ref(const double r[4], R gm1) {
  constexpr int NN = 1 + AX, TT = 2 - AX;
  DevRef<R> c;
  c.rho = (R)r[0];
  c.mn = (R)r[NN];
  c.mt = (R)r[TT];
  const R E = (R)r[3];
  const R ir = recip(c.rho);
  c.un = c.mn * ir;
  c.ut = c.mt * ir;
  c.K = R(0.5) * r_fma(c.mn, c.un, c.mt * c.ut);
  c.p = gm1 * (E - c.K);
  c.H = E + c.p;
  return c;
}

// Full-state values at deviation d from the reference: rho, 1/rho, u_n,
// p, and the deviations du_n and dp the flux deviation uses. The kinetic
// energy K = |m|^2 / (2 rho) changes by
//   dK = ((m_r + dm/2) . dm - K_r drho) / rho,
// which needs no tangential velocity.
template <int AX, typename R>
struct DevState {
  R rho, ir, un, p, dun, dp;
  __device__ __forceinline__ DevState(const R d[4], const DevRef<R>& c, R gm1) {
    constexpr int NN = 1 + AX, TT = 2 - AX;
    rho = c.rho + d[0];
    ir = recip(rho);
    dun = r_fma(-c.un, d[0], d[NN]) * ir;
    un = c.un + dun;
    const R mhn = r_fma(R(0.5), d[NN], c.mn), mht = r_fma(R(0.5), d[TT], c.mt);
    const R dK = r_fma(-c.K, d[0], r_fma(mhn, d[NN], mht * d[TT])) * ir;
    dp = gm1 * (d[3] - dK);
    p = c.p + dp;
  }
};

// dF = F(q_r + d) - F(q_r) for the flux along AX; also the state values.
template <int AX, typename R>
__device__ __forceinline__ DevState<AX, R> dev_flux(const R d[4], const DevRef<R>& c, R gm1,
                                                    R F[4]) {
  constexpr int NN = 1 + AX, TT = 2 - AX;
  const DevState<AX, R> s(d, c, gm1);
  const R dEp = d[3] + s.dp;
  F[0] = d[NN];
  F[NN] = r_fma(c.mn, s.dun, r_fma(d[NN], s.un, s.dp));
  F[TT] = r_fma(c.mt, s.dun, d[TT] * s.un);
  F[3] = r_fma(s.dun, c.H + dEp, c.un * dEp);
  return s;
}

// Rusanov flux in a line's frame: both face states and the result are
// deviations from that line's reference (F_hat - F(q_r)).
template <int AX, typename R>
__device__ __forceinline__ void rusanov_dev(const R dL[4], const R dR[4], const DevRef<R>& c,
                                            R gam, R gm1, R Fh[4], bool& bad) {
  R fL[4], fR[4];
  const DevState<AX, R> sL = dev_flux<AX>(dL, c, gm1, fL);
  const DevState<AX, R> sR = dev_flux<AX>(dR, c, gm1, fR);
  const R lL = fabs(sL.un) + sqrt_pos(gam * sL.p * sL.ir);
  const R lR = fabs(sR.un) + sqrt_pos(gam * sR.p * sR.ir);
  const R lam = (lL >= lR) ? lL : lR;
#pragma unroll
  for (int k = 0; k < 4; ++k) Fh[k] = r_fma(-(R(0.5) * lam), dR[k] - dL[k], R(0.5) * (fL[k] + fR[k]));
  bad = bad || nonphysical(sL.rho, sL.p) || nonphysical(sR.rho, sR.p);
}

// line_ops in deviation form: d the line's deviations; face states and
// face fluxes come back in the line's frame.
template <int N1, int AX, bool LOB, typename R>
__device__ __forceinline__ void line_ops_dev(const R d[4][N1], const DevRef<R>& c,
                                             const KTab<R, N1>& T, R gm1, R qlo[4], R qhi[4],
                                             R flo[4], R fhi[4], R dF[4][N1], bool& bad) {
  R F[4][N1];
#pragma unroll
  for (int n = 0; n < N1; ++n) {
    R dp[4] = {d[0][n], d[1][n], d[2][n], d[3][n]};
    R fp[4];
    const DevState<AX, R> s = dev_flux<AX>(dp, c, gm1, fp);
    bad = bad || nonphysical(s.rho, s.p);
#pragma unroll
    for (int k = 0; k < 4; ++k) F[k][n] = fp[k];
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (LOB) {
      qlo[k] = d[k][0];
      qhi[k] = d[k][N1 - 1];
      flo[k] = F[k][0];
      fhi[k] = F[k][N1 - 1];
    } else {
      qlo[k] = dot_n<N1>([&](int n) { return T.em(n); }, d[k]);
      qhi[k] = dot_n<N1>([&](int n) { return T.ep(n); }, d[k]);
      flo[k] = dot_n<N1>([&](int n) { return T.em(n); }, F[k]);
      fhi[k] = dot_n<N1>([&](int n) { return T.ep(n); }, F[k]);
    }
#pragma unroll
    for (int i = 0; i < N1; ++i) dF[k][i] = dot_n<N1>([&](int n) { return T.D(i, n); }, F[k]);
  }
}

// line_ops_chain in deviation form: D q = D d, and the chain rule's
// coefficients (velocity, pressure, E + p at each point) come from the
// reference plus the deviation.
template <int N1, int AX, typename R>
__device__ __forceinline__ void line_ops_chain_dev(const R d[4][N1], const DevRef<R>& c,
                                                   const KTab<R, N1>& T, R gm1, R qlo[4],
                                                   R qhi[4], R flo[4], R fhi[4], R dF[4][N1],
                                                   bool& bad) {
  constexpr int NN = 1 + AX, TT = 2 - AX;
#pragma unroll
  for (int i = 0; i < N1; ++i) {
    R dq[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) dq[k] = dot_n<N1>([&](int n) { return T.D(i, n); }, d[k]);
    const R dp_[4] = {d[0][i], d[1][i], d[2][i], d[3][i]};
    const DevState<AX, R> s(dp_, c, gm1);
    bad = bad || nonphysical(s.rho, s.p);
    const R ut = c.ut + r_fma(-c.ut, dp_[0], dp_[TT]) * s.ir;
    const R mn = c.mn + dp_[NN], mt = c.mt + dp_[TT];
    const R Ep = c.H + (dp_[3] + s.dp);
    const R dun = r_fma(-s.un, dq[0], dq[NN]) * s.ir;
    const R dp = gm1 * r_fma(R(0.5) * r_fma(s.un, s.un, ut * ut), dq[0],
                             dq[3] - r_fma(s.un, dq[NN], ut * dq[TT]));
    dF[0][i] = dq[NN];
    dF[NN][i] = r_fma(mn, dun, r_fma(dq[NN], s.un, dp));
    dF[TT][i] = r_fma(mt, dun, dq[TT] * s.un);
    dF[3][i] = r_fma(Ep, dun, s.un * (dq[3] + dp));
  }
  R dlo[4], dhi[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    dlo[k] = qlo[k] = d[k][0];
    dhi[k] = qhi[k] = d[k][N1 - 1];
  }
  (void)dev_flux<AX>(dlo, c, gm1, flo);
  (void)dev_flux<AX>(dhi, c, gm1, fhi);
}

// Line operations on the N1 points of one element row (AX=0) or column
// (AX=1): face states qlo (at -1) and qhi (at +1), the flux interpolant's
// face values flo, fhi, and its derivative dF at the points. On Gauss points
// (LOB false) the face values are extrapolated; on Gauss-Lobatto points the
// end points are solution points and the face values are the end values.
template <int N1, int AX, bool LOB, typename R>
__device__ __forceinline__ void line_ops(const R q[4][N1], const KTab<R, N1>& T, R gm1,
                                         R qlo[4], R qhi[4], R flo[4], R fhi[4],
                                         R dF[4][N1], bool& bad) {
  R F[4][N1];
#pragma unroll
  for (int n = 0; n < N1; ++n) {
    R qp[4] = {q[0][n], q[1][n], q[2][n], q[3][n]};
    R fp[4], un, p, ir;
    euler_flux<AX>(qp, gm1, fp, un, p, ir);
    bad = bad || nonphysical(qp[0], p);
#pragma unroll
    for (int k = 0; k < 4; ++k) F[k][n] = fp[k];
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (LOB) {
      qlo[k] = q[k][0];
      qhi[k] = q[k][N1 - 1];
      flo[k] = F[k][0];
      fhi[k] = F[k][N1 - 1];
    } else {
      qlo[k] = dot_n<N1>([&](int n) { return T.em(n); }, q[k]);
      qhi[k] = dot_n<N1>([&](int n) { return T.ep(n); }, q[k]);
      flo[k] = dot_n<N1>([&](int n) { return T.em(n); }, F[k]);
      fhi[k] = dot_n<N1>([&](int n) { return T.ep(n); }, F[k]);
    }
#pragma unroll
    for (int i = 0; i < N1; ++i) dF[k][i] = dot_n<N1>([&](int n) { return T.D(i, n); }, F[k]);
  }
}

// The same line operations for the Gauss-Lobatto scheme with the chain-rule
// divergence (Section 2.2; the CPR flux kernel, Algorithms 7 and 8). The end
// points are solution points, so the face states are the end values and the
// face fluxes the fluxes there; dF at each point is the flux Jacobian applied
// to the derivative of the solution polynomial, A(q) (D q), formed without
// the matrix. With u_n = q_n / rho the velocity along the line, u_t across
// it, and du_n = (dm_n - u_n drho) / rho:
//   dp              = (g-1) (dE + |V|^2/2 drho - (u_n dm_n + u_t dm_t))
//   d(m_n)          = dm_n
//   d(m_n u_n + p)  = dm_n u_n + m_n du_n + dp
//   d(m_t u_n)      = dm_t u_n + m_t du_n
//   d(u_n (E + p))  = du_n (E + p) + u_n (dE + dp)
// Every expression is written in line-normal and line-tangential terms, so
// the two sweeps round identically on transposed data.
template <int N1, int AX, typename R>
__device__ __forceinline__ void line_ops_chain(const R q[4][N1], const KTab<R, N1>& T, R gm1,
                                               R qlo[4], R qhi[4], R flo[4], R fhi[4],
                                               R dF[4][N1], bool& bad) {
  constexpr int NN = 1 + AX, TT = 2 - AX;
#pragma unroll
  for (int i = 0; i < N1; ++i) {
    R dq[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) dq[k] = dot_n<N1>([&](int n) { return T.D(i, n); }, q[k]);
    const R rho = q[0][i], mn = q[NN][i], mt = q[TT][i], E = q[3][i];
    const R ir = recip(rho);
    const R un = mn * ir, ut = mt * ir;
    const R p = gm1 * r_fma(-(R(0.5) * sym_dot2(q[1][i], q[1][i], q[2][i], q[2][i])), ir, E);
    bad = bad || nonphysical(rho, p);
    const R dun = r_fma(-un, dq[0], dq[NN]) * ir;
    const R dp = gm1 * r_fma(R(0.5) * sym_dot2(un, un, ut, ut), dq[0],
                             dq[3] - sym_dot2(un, dq[NN], ut, dq[TT]));
    dF[0][i] = dq[NN];
    dF[NN][i] = r_fma(mn, dun, r_fma(dq[NN], un, dp));
    dF[TT][i] = r_fma(mt, dun, dq[TT] * un);
    dF[3][i] = r_fma(E + p, dun, un * (dq[3] + dp));
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    qlo[k] = q[k][0];
    qhi[k] = q[k][N1 - 1];
  }
  R un, p, ir;
  euler_flux<AX>(qlo, gm1, flo, un, p, ir);
  euler_flux<AX>(qhi, gm1, fhi, un, p, ir);
}

// Coalesced copy between one tile of a state (4 variables x kTile element
// rows, each a contiguous run of nax*NSP float64 in global memory) and its
// LDS image (element stride S). The 4*kTile runs are dealt to the NW waves
// of the workgroup (wave w takes runs w, w+NW, ...); within a run, lane l
// of pass it handles value it*64+l. All loads of a wave are issued before
// any of them is consumed, so one memory round trip covers the whole copy.
// With runs of at least 64 values (PAIRS), 16-byte aligned states and even
// run offsets, a lane moves two neighbouring values per access instead
// (pass it, lane l: values 2(it*64+l) and the next), which halves the
// memory instructions. With an odd number of points per element the two
// may lie in neighbouring elements, so each has its own LDS slot.
template <int N1, int S, int NW = N1>
struct TileCopy {
  static constexpr int NSP = N1 * N1;
  static constexpr int SEG = kTile * NSP;          // values in a full run
  static constexpr int NIT = (SEG + 63) / 64;      // passes per run
  static constexpr int NRUN = (4 * kTile + NW - 1) / NW;  // runs per wave (NW waves)
  // pairs where a run holds at least 64 values (P >= 2); at P = 1 they
  // would leave most lanes idle and cost registers
  static constexpr bool PAIRS = SEG >= 64;
  static constexpr int NIT2 = (SEG / 2 + 63) / 64;  // passes per run, in pairs
  int loff[NIT];    // LDS offset, within its run, of the value a lane moves
  int loff2[NIT2];   // the same for the first value of a lane's pair
  int loff2b[NIT2];  // and for its second
  __device__ __forceinline__ explicit TileCopy(int lane) {
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
      const int f = it * 64 + lane;
      const int cx = f / NSP;
      loff[it] = cx * S + (f - cx * NSP);
    }
#pragma unroll
    for (int it = 0; it < NIT2; ++it) {
      const int f = 2 * (it * 64 + lane);
      const int cx = f / NSP;
      loff2[it] = cx * S + (f - cx * NSP);
      const int cx2 = (f + 1) / NSP;
      loff2b[it] = cx2 * S + (f + 1 - cx2 * NSP);
    }
  }
  // run u of wave wv: variable k, tile row cy; valid when sg < 4*kTile.
  __device__ __forceinline__ static int run(int wv, int u) { return wv + NW * u; }
};

// XCD-aware tile order. Consecutive dispatch slots go round-robin over the
// 8 XCDs. When the row of ngx tile groups splits into 8 equal strips, XCD x
// takes the strip of columns [x sw, (x+1) sw) and walks it row by row: a
// tile's north and south neighbours then pass through the same L2 within a
// row of the strip, and only the strips' side edges cross XCDs. Otherwise
// each XCD takes a contiguous range of the ngx * ngy groups (raster order,
// x fastest). Both maps are permutations of [0, ngx * ngy) for a grid of
// exactly ngx * ngy workgroups.
__device__ __forceinline__ int xcd_tile(int bid, int ngx, int ngy) {
  const int xcd = bid & 7, k = bid >> 3;
  if ((ngx & 7) == 0) {
    const int sw = ngx >> 3;
    return (k / sw) * ngx + xcd * sw + k % sw;
  }
  const int n = ngx * ngy;
  const int per = n >> 3, rem = n & 7;
  return xcd * per + (xcd < rem ? xcd : rem) + k;
}

}  // namespace cpr
