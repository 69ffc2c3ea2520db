// Discrete adjoint of the CPR residual: out = alpha v + delta J(q)^T v +
// beta x + gam y, J = dR/dq of the residual of cpr_stage.hip. The line
// algebra runs in the residual's compute type R (float64, or float32 for the
// FP32-bulk residual); q, v, x, y, out and the combination are float64. In
// float32 the LDS images of q and v are float32 too, which halves the
// kernel's LDS (at P=4: 54 instead of 108 KB, three workgroups per CU
// instead of one), and the epilogue adds alpha v from the float64 state.
//
// Same tile and lane layout as the forward stage kernel: an 8x8 element
// tile per workgroup, wave w on line w of every element. Each line is the
// transpose of the forward 1D CPR operator along it. With a = -(2/h) v on
// the line:
//   sigma_lo = sum_i gL'_i a_i, sigma_hi = sum_i gR'_i a_i   (face flux cotangents)
//   cot f_l  = sum_i D_il a_i - sigma_lo l_l(-1) - sigma_hi l_l(+1)
//   cot q_l  = A(q_l)^T cot f_l + l_l(-1) cot q_lo + l_l(+1) cot q_hi
// where the cotangent of a face flux is the sum of the sigmas of the two
// elements sharing the face, pushed through the transposed Rusanov flux
// (including the derivative of lam = max(|u_n| + c), d|u_n|/du_n = +1 at 0;
// where the two one-sided speeds tie (to 1e-12 relative in float64, 2^-17
// in float32: a tie must be recognised whichever side the rounding of the
// speeds favours, so the threshold sits above that rounding), the gradient of max
// is the mean of both sides' gradients). The two sides' contributions of an interior
// face are exchanged between adjacent lanes by wave shuffles; tile-boundary
// faces are finished by boundary lanes that read the neighbour element's line
// of q and v from global memory. Divisions use the forward kernels'
// reciprocal (hardware estimate and two Newton steps, about 1 ulp). The
// paper (arXiv:1709.01619) has no adjoint; this transposes its Section 2.2
// residual operator.
#include <type_traits>

#include "cpr_device.h"

namespace cpr {

// A number with a first-order perturbation, v + d eps (eps^2 = 0): evaluating
// a function on it gives the function's value and its derivative along d.
template <typename R>
struct Dual {
  R v, d;
};
template <typename R>
__device__ __forceinline__ Dual<R> operator+(Dual<R> a, Dual<R> b) { return {a.v + b.v, a.d + b.d}; }
template <typename R>
__device__ __forceinline__ Dual<R> operator-(Dual<R> a, Dual<R> b) { return {a.v - b.v, a.d - b.d}; }
template <typename R>
__device__ __forceinline__ Dual<R> operator*(Dual<R> a, Dual<R> b) {
  return {a.v * b.v, a.v * b.d + a.d * b.v};
}
template <typename R>
__device__ __forceinline__ Dual<R> operator*(R a, Dual<R> b) { return {a * b.v, a * b.d}; }
template <typename R>
__device__ __forceinline__ Dual<R> operator+(R a, Dual<R> b) { return {a + b.v, b.d}; }
template <typename R>
__device__ __forceinline__ Dual<R> operator-(Dual<R> a) { return {-a.v, -a.d}; }
template <typename R>
__device__ __forceinline__ Dual<R> recip(Dual<R> x) {
  const R r = recip(x.v);
  return {r, -(x.d * r) * r};
}

// (dF_AX/dq)^T s at state q. T is the compute type R, or Dual<R> for the
// derivative of the product along a direction of q (the flux's second
// derivatives contracted with s and that direction).
template <int AX, typename R, typename T = R>
__device__ __forceinline__ void flux_jac_t(const T q[4], R gam, const T s[4], T out[4]) {
  constexpr int n = 1 + AX, t = 2 - AX;
  const T ir = recip(q[0]);
  const T un = q[n] * ir, ut = q[t] * ir;
  const R gm1 = gam - R(1);
  const T ke = R(0.5) * (un * un + ut * ut);
  const T p = gm1 * (q[3] - q[0] * ke);
  const T H = (q[3] + p) * ir;
  const T phi = gm1 * ke;
  out[0] = (phi - un * un) * s[n] - un * ut * s[t] + un * (phi - H) * s[3];
  out[n] = s[0] + (R(3) - gam) * un * s[n] + ut * s[t] + (H - gm1 * un * un) * s[3];
  out[t] = (-gm1) * ut * s[n] + un * s[t] - gm1 * un * ut * s[3];
  out[3] = gm1 * s[n] + gam * un * s[3];
}

// Relative gap below which the two Rusanov speeds count as tied.
__device__ __forceinline__ constexpr double tie_rel(double) { return 1e-12; }
__device__ __forceinline__ constexpr float tie_rel(float) { return 0x1p-17f; }

// Gradient of |u_n| + c with respect to q.
template <int AX, typename R>
__device__ __forceinline__ void wave_speed_grad(const R q[4], R gam, R c, R g[4]) {
  constexpr int n = 1 + AX, t = 2 - AX;
  const R ir = recip(q[0]);
  const R un = q[n] * ir, ut = q[t] * ir;
  const R gg = gam * (gam - R(1));
  const R sgn = un >= R(0) ? R(1) : R(-1);
  const R i2c = R(0.5) * recip(c);
  g[0] = gg * (-q[3] * ir * ir + (un * un + ut * ut) * ir) * i2c - sgn * un * ir;
  g[n] = -gg * un * ir * i2c + sgn * ir;
  g[t] = -gg * ut * ir * i2c;
  g[3] = gg * ir * i2c;
}

// Cotangents of both face states of the Rusanov flux for output cotangent s.
template <int AX, typename R>
__device__ __forceinline__ void rusanov_vjp(const R qL[4], const R qR[4], const R s[4], R gam,
                                            R cL[4], R cR[4], bool& bad) {
  constexpr int n = 1 + AX;
  const R gm1 = gam - R(1);
  const R irL = recip(qL[0]), irR = recip(qR[0]);
  const R pL = gm1 * (qL[3] - R(0.5) * (qL[1] * qL[1] + qL[2] * qL[2]) * irL);
  const R pR = gm1 * (qR[3] - R(0.5) * (qR[1] * qR[1] + qR[2] * qR[2]) * irR);
  const R cLs = sqrt_pos(gam * pL * irL), cRs = sqrt_pos(gam * pR * irR);
  const R lL = fabs(qL[n] * irL) + cLs, lR = fabs(qR[n] * irR) + cRs;
  const R lam = lL >= lR ? lL : lR;
  const bool tie = fabs(lL - lR) <= tie_rel(R(0)) * lam;
  const R wl = tie ? R(0.5) : (lL > lR ? R(1) : R(0));
  const R wr = R(1) - wl;
  R jump = R(0);
#pragma unroll
  for (int k = 0; k < 4; ++k) jump += s[k] * (qR[k] - qL[k]);
  R aL[4], aR[4], gL[4], gR[4];
  flux_jac_t<AX>(qL, gam, s, aL);
  flux_jac_t<AX>(qR, gam, s, aR);
  wave_speed_grad<AX>(qL, gam, cLs, gL);
  wave_speed_grad<AX>(qR, gam, cRs, gR);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    cL[k] = R(0.5) * aL[k] + R(0.5) * lam * s[k] - R(0.5) * jump * wl * gL[k];
    cR[k] = R(0.5) * aR[k] - R(0.5) * lam * s[k] - R(0.5) * jump * wr * gR[k];
  }
  bad = bad || nonphysical(qL[0], pL) || nonphysical(qR[0], pR);
}

template <int N1, int AX, typename R>
struct LineAdj {
  R qlo[4], qhi[4];  // face states
  R slo[4], shi[4];  // own face flux cotangents (sigma)
  R a[4][N1];        // -(2/h) v on the line
};

template <int N1, int AX, typename R>
__device__ __forceinline__ void line_adj_prep(const R q[4][N1], const R v[4][N1],
                                              const KTab<R, N1>& T, R rd,
                                              LineAdj<N1, AX, R>& L) {
#pragma unroll
  for (int k = 0; k < 4; ++k) {
#pragma unroll
    for (int n = 0; n < N1; ++n) L.a[k][n] = rd * v[k][n];
    L.qlo[k] = dot_n<N1>([&](int n) { return T.em(n); }, q[k]);
    L.qhi[k] = dot_n<N1>([&](int n) { return T.ep(n); }, q[k]);
    L.slo[k] = dot_n<N1>([&](int n) { return T.gL(n); }, L.a[k]);
    L.shi[k] = dot_n<N1>([&](int n) { return T.gR(n); }, L.a[k]);
  }
}

// cot q on the line from the face-state cotangents clo, chi.
template <int N1, int AX, typename R>
__device__ __forceinline__ void line_adj_finish(const R q[4][N1], const LineAdj<N1, AX, R>& L,
                                                const R clo[4], const R chi[4],
                                                const KTab<R, N1>& T, R gam, R out[4][N1]) {
#pragma unroll
  for (int l = 0; l < N1; ++l) {
    R cf[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      R s = R(0);
#pragma unroll
      for (int i = 0; i < N1; ++i) s += T.D(i, l) * L.a[k][i];
      cf[k] = s - L.slo[k] * T.em(l) - L.shi[k] * T.ep(l);
    }
    const R qp[4] = {q[0][l], q[1][l], q[2][l], q[3][l]};
    R jt[4];
    flux_jac_t<AX>(qp, gam, cf, jt);
#pragma unroll
    for (int k = 0; k < 4; ++k) out[k][l] = jt[k] + T.em(l) * clo[k] + T.ep(l) * chi[k];
  }
}

// cot q on the line for the chain-rule scheme (Gauss-Lobatto points, the
// paper's CPR). Its divergence A(q_i) d_i, d_i = sum_m D_im q_m, transposes
// into sum_i D_il A(q_i)^T a_i (through d) plus d/dq [a_l . A(q) d_l] at q_l
// (through A), both from one evaluation of A(q)^T a on q_l + eps d_l; the
// flux interpolant's face values are the end points' fluxes, so the sigma
// terms and the face-state cotangents act at the two end points only.
template <int N1, int AX, typename R>
__device__ __forceinline__ void line_adj_finish_chain(const R q[4][N1], const LineAdj<N1, AX, R>& L,
                                                      const R clo[4], const R chi[4],
                                                      const KTab<R, N1>& T, R gam,
                                                      R out[4][N1]) {
  R w[4][N1];
#pragma unroll
  for (int l = 0; l < N1; ++l) {
    Dual<R> qd[4], sd[4], od[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      qd[k] = {q[k][l], dot_n<N1>([&](int m) { return T.D(l, m); }, q[k])};
      sd[k] = {L.a[k][l], R(0)};
    }
    flux_jac_t<AX, R, Dual<R>>(qd, gam, sd, od);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      w[k][l] = od[k].v;    // A(q_l)^T a_l
      out[k][l] = od[k].d;  // d/dq [a_l . A(q) d_l]
    }
  }
#pragma unroll
  for (int l = 0; l < N1; ++l)
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      R acc = out[k][l];
#pragma unroll
      for (int i = 0; i < N1; ++i) acc += T.D(i, l) * w[k][i];
      out[k][l] = acc;
    }
  // end points: the interpolant's face values f(q_0), f(q_N) and the face states
  R ms[4], jt[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) ms[k] = -L.slo[k];
  {
    const R q0[4] = {q[0][0], q[1][0], q[2][0], q[3][0]};
    flux_jac_t<AX, R>(q0, gam, ms, jt);
#pragma unroll
    for (int k = 0; k < 4; ++k) out[k][0] += jt[k] + clo[k];
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) ms[k] = -L.shi[k];
  {
    const R qn[4] = {q[0][N1 - 1], q[1][N1 - 1], q[2][N1 - 1], q[3][N1 - 1]};
    flux_jac_t<AX, R>(qn, gam, ms, jt);
#pragma unroll
    for (int k = 0; k < 4; ++k) out[k][N1 - 1] += jt[k] + chi[k];
  }
}

// One sweep of the transpose along AX for the split layout: the line of
// every element this wave owns (point n of variable k at
// k * VS + base + n * step in the q and v images) is read for its face
// terms, the interior faces are finished with the neighbours by wave
// shuffles (shift lanes apart; hlo / hhi the tile-boundary face-state
// cotangents where at_lo / at_hi), and the line is read again for the
// interior transpose, whose values go to emit(k, n, value).
template <int N1, int AX, bool CHAIN, typename R, typename LT, typename Emit>
__device__ __forceinline__ void adj_sweep_split(const LT* qs, const LT* vs, int VS, int base,
                                                int step, const KTab<R, N1>& T, R rd, R gam,
                                                int shift, bool at_lo, bool at_hi, const R* hlo,
                                                const R* hhi, bool act, bool& bad, Emit emit) {
  R qlo[4], qhi[4], slo[4], shi[4];
  {
    R q[4][N1], v[4][N1];
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
      for (int n = 0; n < N1; ++n) {
        q[k][n] = (R)qs[k * VS + base + n * step];
        v[k][n] = (R)vs[k * VS + base + n * step];
      }
    LineAdj<N1, AX, R> L;
    line_adj_prep<N1, AX>(q, v, T, rd, L);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      qlo[k] = L.qlo[k];
      qhi[k] = L.qhi[k];
      slo[k] = L.slo[k];
      shi[k] = L.shi[k];
    }
  }
  // the line is read again below rather than kept across the Rusanov
  // transpose
  asm volatile("" ::: "memory");
  R qnb[4], s[4], cL[4], cR[4], clo[4], chi[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    qnb[k] = __shfl_up(qhi[k], shift, 64);
    s[k] = slo[k] + __shfl_up(shi[k], shift, 64);
  }
  bool b2 = false;
  rusanov_vjp<AX>(qnb, qlo, s, gam, cL, cR, b2);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    clo[k] = cR[k];
    chi[k] = __shfl_down(cL[k], shift, 64);
  }
  if (at_lo) {
#pragma unroll
    for (int k = 0; k < 4; ++k) clo[k] = hlo[k];
    b2 = false;
  }
  if (at_hi) {
#pragma unroll
    for (int k = 0; k < 4; ++k) chi[k] = hhi[k];
  }
  if (act) bad = bad || b2;
  R q[4][N1], v[4][N1], out[4][N1];
#pragma unroll
  for (int k = 0; k < 4; ++k)
#pragma unroll
    for (int n = 0; n < N1; ++n) {
      q[k][n] = (R)qs[k * VS + base + n * step];
      v[k][n] = (R)vs[k * VS + base + n * step];
    }
  LineAdj<N1, AX, R> L;
  line_adj_prep<N1, AX>(q, v, T, rd, L);
  if constexpr (CHAIN)
    line_adj_finish_chain<N1, AX>(q, L, clo, chi, T, gam, out);
  else
    line_adj_finish<N1, AX>(q, L, clo, chi, T, gam, out);
#pragma unroll
  for (int k = 0; k < 4; ++k)
#pragma unroll
    for (int n = 0; n < N1; ++n) emit(k, n, out[k][n]);
}

// Third-image layout with concurrent sweeps: P=4 in float64 with the flux
// derivative (see the kernel); the chain rule's dual-number transpose needs
// more registers than three waves per SIMD leave.
template <int P, typename R, bool CHAIN>
struct VjpSplit {
  static constexpr bool value = sizeof(R) == 8 && P == 4 && !CHAIN;
};

template <int P, typename R, bool CHAIN>
__global__ __launch_bounds__((64 * (VjpSplit<P, R, CHAIN>::value ? 2 * (P + 1) : P + 1)),
                             (VjpSplit<P, R, CHAIN>::value ? 3 : 1)) void vjp_kernel(
    Geometry G, KTab<R, P + 1> T, VjpArgs A) {
  constexpr int N1 = P + 1;
  constexpr int NSP = N1 * N1;
  constexpr int S = (NSP & 1) ? NSP : NSP + 1;
  // P=4 in float64 (split layout): the q and v images of a tile take
  // 105 KB, so a CU holds one workgroup either way. A third image takes the
  // column results (155 KB in all), which lets the column sweep (the first
  // P+1 waves) and the row sweep (the next P+1) run at the same time, neither
  // overwriting an image the other reads; each sweep reads its line twice
  // from LDS (face terms, then interior) rather than holding it across the
  // Rusanov transpose, which keeps the registers within three waves per
  // SIMD. Measured and not kept, at P=4 1024^2: half-height tiles with two
  // lines per wave and two workgroups per CU (1.75 ms per launch against
  // 1.20 ms: twice the tile-boundary work, and register spills); direct
  // global-to-LDS copies of q and v (3 % slower than the register-staged
  // pairs); and one workgroup per CU walking its share of the tiles with the
  // next tile's copies in flight during the epilogue (5 % slower: its wait
  // for the copies also waits for the last tile's stores, which a finished
  // workgroup leaves to drain).
  constexpr bool OIMG = VjpSplit<P, R, CHAIN>::value;
  constexpr int NW = OIMG ? 2 * N1 : N1;  // waves per workgroup
  constexpr int VS = 64 * S;
  // LDS images in the compute type: float64 states are rounded to float32
  // here in FP32-bulk, as the line algebra does anyway
  using LT = R;
  constexpr bool F32 = sizeof(R) == 4;
  __shared__ LT qs[4 * VS];
  __shared__ LT vs[4 * VS];
  // inside face-state cotangents at tile boundaries: W, E and S, N
  __shared__ R hCx[2][kTile][N1][4];
  __shared__ R hCy[2][kTile][N1][4];
  __shared__ LT os_img[OIMG ? 4 * VS : 1];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform
  const int tile = xcd_tile(blockIdx.x, G.ntx, G.nty);
  const int tx = tile % G.ntx, ty = tile / G.ntx;
  const int I0 = tx * kTile, J0 = ty * kTile;
  const int nax = min(kTile, G.nx - I0), nay = min(kTile, G.ny - J0);
  const size_t plane = (size_t)G.ny * G.nx * NSP;
  const R gam = T.gam;
  const R rdx = T.rdx, rdy = T.rdy;
  bool bad = false;

  // tile of q and of v -> LDS; each wave issues all its loads of an array
  // before writing any of them. In the split layout the loads of both
  // arrays go out together (one memory round trip instead of two, at no
  // cost in the register peak, which the sweeps set): 1.13 -> 1.07 ms per
  // launch at P=4 1024^2. With three float32-image workgroups per CU the
  // same order measured 42 % slower, so the other layouts copy q, then v.
  using TC = TileCopy<N1, S, NW>;
  const TC tc(lane);
  const int seg_len = nax * NSP;
  // paired 16-byte copies of q, v, x, y and out (float64 states in both
  // precisions), on the same conditions as in the stage kernel (aligned
  // states, even run offsets, whole pairs); this kernel's LDS already holds
  // it to one or two workgroups per CU, so the pair registers cost nothing
  constexpr bool PAIRS = TC::PAIRS;
  const bool pairs_ok = A.vec && (NSP % 2 == 0 || (G.nx % 2 == 0 && seg_len % 2 == 0));
  constexpr int NA = OIMG ? 2 : 1;  // arrays whose loads are in flight together
  const auto src_of = [&](int arr) { return arr == 0 ? A.q : A.v; };
  const auto lds_of = [&](int arr) { return arr == 0 ? qs : vs; };
#pragma unroll
  for (int a0 = 0; a0 < 2; a0 += NA) {
    if (PAIRS && pairs_ok) {
      double2 t2[NA][TC::NRUN][TC::NIT2];
#pragma unroll
      for (int j = 0; j < NA; ++j)
#pragma unroll
        for (int u = 0; u < TC::NRUN; ++u) {
          const int sg = TC::run(wv, u);
          const int k = sg >> 3, cy = sg & 7;
          const bool ok = sg < 4 * kTile && cy < nay;
          const double* src = src_of(a0 + j) + k * plane + ((size_t)(J0 + cy) * G.nx + I0) * NSP;
#pragma unroll
          for (int it = 0; it < TC::NIT2; ++it) {
            const int f = 2 * (it * 64 + lane);
            if (ok && f < seg_len) t2[j][u][it] = *reinterpret_cast<const double2*>(src + f);
          }
        }
#pragma unroll
      for (int j = 0; j < NA; ++j)
#pragma unroll
        for (int u = 0; u < TC::NRUN; ++u) {
          const int sg = TC::run(wv, u);
          const int k = sg >> 3, cy = sg & 7;
          const bool ok = sg < 4 * kTile && cy < nay;
          LT* dst = lds_of(a0 + j) + k * VS + cy * kTile * S;
#pragma unroll
          for (int it = 0; it < TC::NIT2; ++it) {
            const int f = 2 * (it * 64 + lane);
            if (ok && f < seg_len) {
              dst[tc.loff2[it]] = (LT)t2[j][u][it].x;
              dst[tc.loff2b[it]] = (LT)t2[j][u][it].y;
            }
          }
        }
      continue;
    }
    double t[NA][TC::NRUN][TC::NIT];
#pragma unroll
    for (int j = 0; j < NA; ++j)
#pragma unroll
      for (int u = 0; u < TC::NRUN; ++u) {
        const int sg = TC::run(wv, u);
        const int k = sg >> 3, cy = sg & 7;
        const bool ok = sg < 4 * kTile && cy < nay;
        const double* src = src_of(a0 + j) + k * plane + ((size_t)(J0 + cy) * G.nx + I0) * NSP;
#pragma unroll
        for (int it = 0; it < TC::NIT; ++it) {
          const int f = it * 64 + lane;
          t[j][u][it] = (ok && f < seg_len) ? src[f] : 0.0;
        }
      }
#pragma unroll
    for (int j = 0; j < NA; ++j)
#pragma unroll
      for (int u = 0; u < TC::NRUN; ++u) {
        const int sg = TC::run(wv, u);
        const int k = sg >> 3, cy = sg & 7;
        const bool ok = sg < 4 * kTile && cy < nay;
        LT* dst = lds_of(a0 + j) + k * VS + cy * kTile * S;
#pragma unroll
        for (int it = 0; it < TC::NIT; ++it) {
          const int f = it * 64 + lane;
          if (ok && f < seg_len) dst[tc.loff[it]] = (LT)t[j][u][it];
        }
      }
  }

  const bool halo = tid < 4 * kTile * N1;
  int hs = 0, hp = 0, hm = 0;
  bool hact = false, hout = false;
  R oq[4] = {R(0), R(0), R(0), R(0)}, os[4] = {R(0), R(0), R(0), R(0)};
  if (halo) {
    hs = tid / (kTile * N1);
    const int r2 = tid - hs * (kTile * N1);
    hp = r2 / N1;
    hm = r2 - hp * N1;
    int Io, Jo;
    if (hs < 2) {
      hact = hp < nay;
      Jo = J0 + hp;
      Io = (hs == 0) ? I0 - 1 : I0 + nax;
    } else {
      hact = hp < nax;
      Io = I0 + hp;
      Jo = (hs == 2) ? J0 - 1 : J0 + nay;
    }
    hout = true;
    if (Io < 0 || Io >= G.nx) {
      if (G.periodic) Io = (Io + G.nx) % G.nx; else hout = false;
    }
    if (Jo < 0 || Jo >= G.ny) {
      if (G.periodic) Jo = (Jo + G.ny) % G.ny; else hout = false;
    }
    if (hact && hout) {
      const size_t base = ((size_t)Jo * G.nx + Io) * NSP;
      R lq[4][N1], la[4][N1];
      const R rd = hs < 2 ? rdx : rdy;
#pragma unroll
      for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int n = 0; n < N1; ++n) {
          const size_t g = k * plane + base + (hs < 2 ? hm * N1 + n : n * N1 + hm);
          lq[k][n] = (R)A.q[g];
          la[k][n] = rd * (R)A.v[g];
        }
      // the outside element's face that touches this tile
      const bool hi_face = (hs == 0 || hs == 2);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        oq[k] = dot_n<N1>([&](int n) { return hi_face ? T.ep(n) : T.em(n); }, lq[k]);
        os[k] = dot_n<N1>([&](int n) { return hi_face ? T.gR(n) : T.gL(n); }, la[k]);
      }
    }
  }
  __syncthreads();

  if (halo && hact) {
    int e, stride, off;
    if (hs < 2) {
      e = hp * kTile + (hs == 0 ? 0 : nax - 1);
      off = hm * N1;
      stride = 1;
    } else {
      e = (hs == 2 ? 0 : nay - 1) * kTile + hp;
      off = hm;
      stride = N1;
    }
    const R rd = hs < 2 ? rdx : rdy;
    R lq[4][N1], la[4][N1];
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
      for (int n = 0; n < N1; ++n) {
        lq[k][n] = (R)qs[k * VS + e * S + off + n * stride];
        la[k][n] = rd * (R)vs[k * VS + e * S + off + n * stride];
      }
    const bool lo_side = (hs == 0 || hs == 2);  // this tile's face is its low face
    R iq[4], is[4], s[4], qL[4], qR[4], cL[4], cR[4], cin[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      iq[k] = dot_n<N1>([&](int n) { return lo_side ? T.em(n) : T.ep(n); }, lq[k]);
      is[k] = dot_n<N1>([&](int n) { return lo_side ? T.gL(n) : T.gR(n); }, la[k]);
      if (!hout) oq[k] = iq[k];
      s[k] = hout ? is[k] + os[k] : is[k];
      qL[k] = lo_side ? oq[k] : iq[k];
      qR[k] = lo_side ? iq[k] : oq[k];
    }
    if (hs < 2)
      rusanov_vjp<0>(qL, qR, s, gam, cL, cR, bad);
    else
      rusanov_vjp<1>(qL, qR, s, gam, cL, cR, bad);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      // transmissive: both face states are the inside state
      cin[k] = !hout ? cL[k] + cR[k] : (lo_side ? cR[k] : cL[k]);
      if (hs < 2)
        hCx[hs][hp][hm][k] = cin[k];
      else
        hCy[hs - 2][hp][hm][k] = cin[k];
    }
  }

  // one lane -> element map for both sweeps: x neighbours are 1 lane
  // apart, y neighbours 8 lanes apart
  const int cxX = lane & 7, cyX = lane >> 3, eX = lane;
  const int cxY = lane & 7, cyY = lane >> 3, eY = lane;
  const bool actX = cxX < nax && cyX < nay;
  const bool actY = cxY < nax && cyY < nay;
  LT* const oimg = OIMG ? os_img : qs;

  if constexpr (OIMG) {
    __syncthreads();  // images and tile-boundary cotangents are in LDS
    const int grp = wv >= N1 ? 1 : 0;  // wave-uniform: 0 column sweep, 1 row sweep
    const int ln = wv - grp * N1;       // the line of every element this wave takes
    const int el = lane, cx = lane & 7, cy = lane >> 3;
    const bool act = cx < nax && cy < nay;
    // the row sweep keeps its results in registers until the column
    // results are in the third image, then each row lane combines its own
    // points
    R orow[4][N1];
    if (grp == 0)
      adj_sweep_split<N1, 1, CHAIN>(qs, vs, VS, el * S + ln, N1, T, rdy, gam, kTile, cy == 0,
                                    cy == nay - 1, hCy[0][cx][ln], hCy[1][cx][ln], act, bad,
                                    [&](int k, int n, R v) { os_img[k * VS + el * S + n * N1 + ln] = v; });
    else
      adj_sweep_split<N1, 0, CHAIN>(qs, vs, VS, el * S + ln * N1, 1, T, rdx, gam, 1, cx == 0,
                                    cx == nax - 1, hCx[0][cy][ln], hCx[1][cy][ln], act, bad,
                                    [&](int k, int n, R v) { orow[k][n] = v; });
    __syncthreads();  // every column result is in the third image
    if (grp == 1) {
#pragma unroll
      for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int n = 0; n < N1; ++n) {
          const int a = k * VS + el * S + ln * N1 + n;
          os_img[a] = A.alpha * vs[a] + A.delta * ((double)orow[k][n] + os_img[a]);
        }
    }
  } else {
  // Each sweep holds only its own line: the column sweep's result stays in
  // registers until every lane has read its row, then replaces q in LDS.
  R qcol[4][N1], vcol[4][N1];
#pragma unroll
  for (int k = 0; k < 4; ++k)
#pragma unroll
    for (int n = 0; n < N1; ++n) {
      qcol[k][n] = (R)qs[k * VS + eY * S + n * N1 + wv];
      vcol[k][n] = (R)vs[k * VS + eY * S + n * N1 + wv];
    }
  __syncthreads();  // tile-boundary cotangents are in hC

  // ---- column sweep (y) ----
  R oc[4][N1];
  {
    LineAdj<N1, 1, R> L;
    line_adj_prep<N1, 1>(qcol, vcol, T, rdy, L);
    R qnb[4], snb[4], s[4], cL[4], cR[4], clo[4], chi[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      qnb[k] = __shfl_up(L.qhi[k], kTile, 64);
      snb[k] = __shfl_up(L.shi[k], kTile, 64);
      s[k] = L.slo[k] + snb[k];
    }
    bool b2 = false;
    rusanov_vjp<1>(qnb, L.qlo, s, gam, cL, cR, b2);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      clo[k] = cR[k];
      chi[k] = __shfl_down(cL[k], kTile, 64);
    }
    if (cyY == 0) {
#pragma unroll
      for (int k = 0; k < 4; ++k) clo[k] = hCy[0][cxY][wv][k];
      b2 = false;
    }
    if (cyY == nay - 1) {
#pragma unroll
      for (int k = 0; k < 4; ++k) chi[k] = hCy[1][cxY][wv][k];
    }
    if constexpr (CHAIN)
      line_adj_finish_chain<N1, 1>(qcol, L, clo, chi, T, gam, oc);
    else
      line_adj_finish<N1, 1>(qcol, L, clo, chi, T, gam, oc);
    if (actY) bad = bad || b2;
  }

  R qrow[4][N1], vrow[4][N1];
#pragma unroll
  for (int k = 0; k < 4; ++k)
#pragma unroll
    for (int n = 0; n < N1; ++n) {
      qrow[k][n] = (R)qs[k * VS + eX * S + wv * N1 + n];
      vrow[k][n] = (R)vs[k * VS + eX * S + wv * N1 + n];
    }
  __syncthreads();  // every row has been read
#pragma unroll
  for (int k = 0; k < 4; ++k)
#pragma unroll
    for (int n = 0; n < N1; ++n) qs[k * VS + eY * S + n * N1 + wv] = (LT)oc[k][n];

  // ---- row sweep (x) ----
  R orow[4][N1];
  {
    LineAdj<N1, 0, R> L;
    line_adj_prep<N1, 0>(qrow, vrow, T, rdx, L);
    R qnb[4], snb[4], s[4], cL[4], cR[4], clo[4], chi[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      qnb[k] = __shfl_up(L.qhi[k], 1, 64);
      snb[k] = __shfl_up(L.shi[k], 1, 64);
      s[k] = L.slo[k] + snb[k];
    }
    bool b2 = false;
    rusanov_vjp<0>(qnb, L.qlo, s, gam, cL, cR, b2);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      clo[k] = cR[k];
      chi[k] = __shfl_down(cL[k], 1, 64);
    }
    if (cxX == 0) {
#pragma unroll
      for (int k = 0; k < 4; ++k) clo[k] = hCx[0][cyX][wv][k];
      b2 = false;
    }
    if (cxX == nax - 1) {
#pragma unroll
      for (int k = 0; k < 4; ++k) chi[k] = hCx[1][cyX][wv][k];
    }
    if constexpr (CHAIN)
      line_adj_finish_chain<N1, 0>(qrow, L, clo, chi, T, gam, orow);
    else
      line_adj_finish<N1, 0>(qrow, L, clo, chi, T, gam, orow);
    if (actX) bad = bad || b2;
  }
  __syncthreads();

#pragma unroll
  for (int k = 0; k < 4; ++k)
#pragma unroll
    for (int n = 0; n < N1; ++n) {
      const int a = k * VS + eX * S + wv * N1 + n;
      if constexpr (F32) {
        qs[a] = orow[k][n] + qs[a];  // J^T v; alpha v and delta follow in float64
      } else {
        // the v image is intact (the column results replaced the q image)
        const double jt = (double)orow[k][n] + qs[a];
        qs[a] = A.alpha * vs[a] + A.delta * jt;
      }
    }
  }
  __syncthreads();

  if constexpr (F32) {
    // FP32-bulk epilogue: out = alpha v + delta (J^T v) + beta x + gam y in
    // float64, the float64 inputs one array at a time (all of an array's
    // loads issued, then accumulated), so that at most two arrays of a
    // wave's values are live; every load precedes the first store (out may
    // alias x)
    if (PAIRS && pairs_ok) {
      double2 ov[TC::NRUN][TC::NIT2], t[TC::NRUN][TC::NIT2];
#pragma unroll
      for (int u = 0; u < TC::NRUN; ++u) {
        const int sg = TC::run(wv, u);
        const int k = sg >> 3, cy = sg & 7;
        const bool ok = sg < 4 * kTile && cy < nay;
        const LT* img = qs + k * VS + cy * kTile * S;
#pragma unroll
        for (int it = 0; it < TC::NIT2; ++it) {
          const int f = 2 * (it * 64 + lane);
          ov[u][it] = (ok && f < seg_len) ? double2{(double)img[tc.loff2[it]], (double)img[tc.loff2b[it]]}
                                          : double2{0.0, 0.0};
        }
      }
#pragma unroll
      for (int arr = 0; arr < 3; ++arr) {
        const double* src = arr == 0 ? A.v : (arr == 1 ? A.x : A.y);
        if (src == nullptr) continue;
#pragma unroll
        for (int u = 0; u < TC::NRUN; ++u) {
          const int sg = TC::run(wv, u);
          const int k = sg >> 3, cy = sg & 7;
          const bool ok = sg < 4 * kTile && cy < nay;
          const size_t gb = k * plane + ((size_t)(J0 + cy) * G.nx + I0) * NSP;
#pragma unroll
          for (int it = 0; it < TC::NIT2; ++it) {
            const int f = 2 * (it * 64 + lane);
            t[u][it] = (ok && f < seg_len) ? *reinterpret_cast<const double2*>(src + gb + f)
                                           : double2{0.0, 0.0};
          }
        }
#pragma unroll
        for (int u = 0; u < TC::NRUN; ++u)
#pragma unroll
          for (int it = 0; it < TC::NIT2; ++it) {
            if (arr == 0) {
              ov[u][it].x = A.alpha * t[u][it].x + A.delta * ov[u][it].x;
              ov[u][it].y = A.alpha * t[u][it].y + A.delta * ov[u][it].y;
            } else {
              const double c = arr == 1 ? A.beta : A.gam;
              ov[u][it].x += c * t[u][it].x;
              ov[u][it].y += c * t[u][it].y;
            }
          }
      }
      __builtin_amdgcn_s_waitcnt(0);
#pragma unroll
      for (int u = 0; u < TC::NRUN; ++u) {
        const int sg = TC::run(wv, u);
        const int k = sg >> 3, cy = sg & 7;
        const bool ok = sg < 4 * kTile && cy < nay;
        const size_t gb = k * plane + ((size_t)(J0 + cy) * G.nx + I0) * NSP;
#pragma unroll
        for (int it = 0; it < TC::NIT2; ++it) {
          const int f = 2 * (it * 64 + lane);
          if (ok && f < seg_len) *reinterpret_cast<double2*>(A.out + gb + f) = ov[u][it];
        }
      }
    } else {
      double ov[TC::NRUN][TC::NIT], t[TC::NRUN][TC::NIT];
#pragma unroll
      for (int u = 0; u < TC::NRUN; ++u) {
        const int sg = TC::run(wv, u);
        const int k = sg >> 3, cy = sg & 7;
        const bool ok = sg < 4 * kTile && cy < nay;
        const LT* img = qs + k * VS + cy * kTile * S;
#pragma unroll
        for (int it = 0; it < TC::NIT; ++it) {
          const int f = it * 64 + lane;
          ov[u][it] = (ok && f < seg_len) ? (double)img[tc.loff[it]] : 0.0;
        }
      }
#pragma unroll
      for (int arr = 0; arr < 3; ++arr) {
        const double* src = arr == 0 ? A.v : (arr == 1 ? A.x : A.y);
        if (src == nullptr) continue;
#pragma unroll
        for (int u = 0; u < TC::NRUN; ++u) {
          const int sg = TC::run(wv, u);
          const int k = sg >> 3, cy = sg & 7;
          const bool ok = sg < 4 * kTile && cy < nay;
          const size_t gb = k * plane + ((size_t)(J0 + cy) * G.nx + I0) * NSP;
#pragma unroll
          for (int it = 0; it < TC::NIT; ++it) {
            const int f = it * 64 + lane;
            t[u][it] = (ok && f < seg_len) ? src[gb + f] : 0.0;
          }
        }
#pragma unroll
        for (int u = 0; u < TC::NRUN; ++u)
#pragma unroll
          for (int it = 0; it < TC::NIT; ++it) {
            if (arr == 0)
              ov[u][it] = A.alpha * t[u][it] + A.delta * ov[u][it];
            else
              ov[u][it] += (arr == 1 ? A.beta : A.gam) * t[u][it];
          }
      }
      __builtin_amdgcn_s_waitcnt(0);
#pragma unroll
      for (int u = 0; u < TC::NRUN; ++u) {
        const int sg = TC::run(wv, u);
        const int k = sg >> 3, cy = sg & 7;
        const bool ok = sg < 4 * kTile && cy < nay;
        const size_t gb = k * plane + ((size_t)(J0 + cy) * G.nx + I0) * NSP;
#pragma unroll
        for (int it = 0; it < TC::NIT; ++it) {
          const int f = it * 64 + lane;
          if (ok && f < seg_len) A.out[gb + f] = ov[u][it];
        }
      }
    }
  } else {
    // epilogue: the x and y loads of a wave are issued before its stores
    // (out may alias x)
    if (PAIRS && pairs_ok) {
      double2 xv[TC::NRUN][TC::NIT2], yv[TC::NRUN][TC::NIT2];
  #pragma unroll
      for (int u = 0; u < TC::NRUN; ++u) {
        const int sg = TC::run(wv, u);
        const int k = sg >> 3, cy = sg & 7;
        const bool ok = sg < 4 * kTile && cy < nay;
        const size_t gb = k * plane + ((size_t)(J0 + cy) * G.nx + I0) * NSP;
  #pragma unroll
        for (int it = 0; it < TC::NIT2; ++it) {
          const int f = 2 * (it * 64 + lane);
          const bool in = ok && f < seg_len;
          xv[u][it] = (in && A.x != nullptr) ? *reinterpret_cast<const double2*>(A.x + gb + f)
                                             : double2{0.0, 0.0};
          yv[u][it] = (in && A.y != nullptr) ? *reinterpret_cast<const double2*>(A.y + gb + f)
                                             : double2{0.0, 0.0};
        }
      }
  #pragma unroll
      for (int u = 0; u < TC::NRUN; ++u) {
        const int sg = TC::run(wv, u);
        const int k = sg >> 3, cy = sg & 7;
        const bool ok = sg < 4 * kTile && cy < nay;
        const double* img = oimg + k * VS + cy * kTile * S;
  #pragma unroll
        for (int it = 0; it < TC::NIT2; ++it) {
          const int f = 2 * (it * 64 + lane);
          if (ok && f < seg_len) {
            double o0 = img[tc.loff2[it]], o1 = img[tc.loff2b[it]];
            if (A.x != nullptr) {
              o0 += A.beta * xv[u][it].x;
              o1 += A.beta * xv[u][it].y;
            }
            if (A.y != nullptr) {
              o0 += A.gam * yv[u][it].x;
              o1 += A.gam * yv[u][it].y;
            }
            xv[u][it] = double2{o0, o1};
          }
        }
      }
      __builtin_amdgcn_s_waitcnt(0);
  #pragma unroll
      for (int u = 0; u < TC::NRUN; ++u) {
        const int sg = TC::run(wv, u);
        const int k = sg >> 3, cy = sg & 7;
        const bool ok = sg < 4 * kTile && cy < nay;
        const size_t gb = k * plane + ((size_t)(J0 + cy) * G.nx + I0) * NSP;
  #pragma unroll
        for (int it = 0; it < TC::NIT2; ++it) {
          const int f = 2 * (it * 64 + lane);
          if (ok && f < seg_len) *reinterpret_cast<double2*>(A.out + gb + f) = xv[u][it];
        }
      }
    } else {
      double xv[TC::NRUN][TC::NIT], yv[TC::NRUN][TC::NIT];
  #pragma unroll
      for (int u = 0; u < TC::NRUN; ++u) {
        const int sg = TC::run(wv, u);
        const int k = sg >> 3, cy = sg & 7;
        const bool ok = sg < 4 * kTile && cy < nay;
        const size_t gb = k * plane + ((size_t)(J0 + cy) * G.nx + I0) * NSP;
  #pragma unroll
        for (int it = 0; it < TC::NIT; ++it) {
          const int f = it * 64 + lane;
          const bool in = ok && f < seg_len;
          xv[u][it] = (in && A.x != nullptr) ? A.x[gb + f] : 0.0;
          yv[u][it] = (in && A.y != nullptr) ? A.y[gb + f] : 0.0;
        }
      }
      // every output value is formed before the first store (see the stage
      // kernel's epilogue), then one explicit wait, then the stores
  #pragma unroll
      for (int u = 0; u < TC::NRUN; ++u) {
        const int sg = TC::run(wv, u);
        const int k = sg >> 3, cy = sg & 7;
        const bool ok = sg < 4 * kTile && cy < nay;
        const double* img = oimg + k * VS + cy * kTile * S;
  #pragma unroll
        for (int it = 0; it < TC::NIT; ++it) {
          const int f = it * 64 + lane;
          if (ok && f < seg_len) {
            double o = img[tc.loff[it]];
            if (A.x != nullptr) o += A.beta * xv[u][it];
            if (A.y != nullptr) o += A.gam * yv[u][it];
            xv[u][it] = o;
          }
        }
      }
      __builtin_amdgcn_s_waitcnt(0);
  #pragma unroll
      for (int u = 0; u < TC::NRUN; ++u) {
        const int sg = TC::run(wv, u);
        const int k = sg >> 3, cy = sg & 7;
        const bool ok = sg < 4 * kTile && cy < nay;
        const size_t gb = k * plane + ((size_t)(J0 + cy) * G.nx + I0) * NSP;
  #pragma unroll
        for (int it = 0; it < TC::NIT; ++it) {
          const int f = it * 64 + lane;
          if (ok && f < seg_len) A.out[gb + f] = xv[u][it];
        }
      }
    }
  }
  if (bad) atomicOr(A.err, 1);
}

template <int P, typename R>
static hipError_t launch_vjp_t(const Geometry& g, const Tables1D& T, const VjpArgs& a,
                               bool chain, hipStream_t s) {
  const KTab<R, P + 1> kt = make_ktab<R, P + 1>(T, g);
  // the split layout (VjpSplit) runs both sweeps at once on 2 (P+1) waves;
  // the plain one runs them in turn on P+1 waves
  const auto launch = [&](auto kernel, bool split) {
    hipLaunchKernelGGL(kernel, dim3(g.ntx * g.nty), dim3(64 * (split ? 2 * (P + 1) : P + 1)), 0, s,
                       g, kt, a);
  };
  if (chain)
    launch(vjp_kernel<P, R, true>, VjpSplit<P, R, true>::value);
  else
    launch(vjp_kernel<P, R, false>, VjpSplit<P, R, false>::value);
  return hipGetLastError();
}

hipError_t launch_vjp(int P, bool fp32, int scheme, const Geometry& g, const Tables1D& T,
                      const VjpArgs& a, hipStream_t s) {
  // the chain-rule transpose takes the face values at the end points, so it
  // needs the Gauss-Lobatto tables
  if (T.points != scheme_points(scheme)) return hipErrorInvalidValue;
  const bool c = scheme == kSchemeGllChain;
  switch (P) {
    case 1: return fp32 ? launch_vjp_t<1, float>(g, T, a, c, s) : launch_vjp_t<1, double>(g, T, a, c, s);
    case 2: return fp32 ? launch_vjp_t<2, float>(g, T, a, c, s) : launch_vjp_t<2, double>(g, T, a, c, s);
    case 3: return fp32 ? launch_vjp_t<3, float>(g, T, a, c, s) : launch_vjp_t<3, double>(g, T, a, c, s);
    case 4: return fp32 ? launch_vjp_t<4, float>(g, T, a, c, s) : launch_vjp_t<4, double>(g, T, a, c, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace cpr
