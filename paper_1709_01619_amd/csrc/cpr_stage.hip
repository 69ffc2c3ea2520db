// Fused CPR residual + SSP-RK3 stage kernel for gfx950.
//
// A tile of 8x8 elements is worked on by 64*(P+1) lanes: wave w works on
// line w of every element of the tile (row w in the x sweep, column w in
// the y sweep), one element per lane. The residual of Section 2.2
// (arXiv:1709.01619) splits into an x part that depends only on element rows
// and a y part that depends only on element columns; each is a 1D CPR
// operator along that line:
//   R = -(2/dx)[D f + (F_W - f_W) gL' + (F_E - f_E) gR']      (rows)
//       -(2/dy)[D g + (G_S - g_S) gL' + (G_N - g_N) gR']      (columns)
// with face states extrapolated from each element's polynomial and the
// Rusanov common flux (Section 4) at every face point.
//
// SCH selects the discretisation. On Gauss-Lobatto points (the paper's CPR,
// Section 2.2 and the CPR flux kernel of Algorithms 7 and 8, and its NDG,
// Section 2.4) face states are end values, so a neighbour contributes one
// point per line; the paper's CPR also replaces D f by the chain rule
// A(q) (D q) (line_ops_chain).
//
// A workgroup holds TPW tiles side by side; the tiles share only the
// barriers. With P = 4 in float64 a one-tile workgroup has 5 waves and
// needs more than 128 VGPRs per lane, and a CU then hosts only one such
// workgroup at a time; a two-tile workgroup (10 waves) keeps two tiles in
// flight per CU.
//
// Phases of one tile:
//  A  the tile (4 variables x 64 elements x (P+1)^2 float64) is copied into
//     LDS with coalesced loads; lanes 0..32(P+1)-1 also load the line of the
//     neighbouring element across the tile boundary that they own. All of
//     a wave's copy loads are issued before any is used: one memory round
//     trip. The scattered neighbour-line loads go out with them, or in
//     float64 from P = 2 just after the copies are in LDS;
//  B  those lanes finish the Rusanov flux on the tile-boundary faces; every
//     lane reads its column out of LDS;
//  C  column sweep: interior face states travel between lanes by wave
//     shuffles (neighbours along a column are 8 lanes apart). The column
//     residual stays in registers until every lane has read its row, then
//     replaces the tile image in LDS;
//  D  row sweep the same way; this tile's q_n loads are issued, then the two
//     parts are summed and the RK combination b (q_src + dt R) is formed in
//     float64 and parked in LDS;
//  E  coalesced epilogue q_dst = a q_n + (parked value). When the limiter
//     follows the stage, the output also stays in LDS and the element means
//     the limiter needs are formed from it, which saves the limiter its own
//     pass over the state.
// Each line is held in registers only during its own sweep, which keeps the
// register peak low enough for several workgroups per CU. Each
// tile-boundary face flux is computed by both tiles that share it from
// bit-identical inputs, so the scheme stays exactly conservative.
#include "cpr_device.h"

namespace cpr {

template <int N1, typename R>
struct TilesPerGroup {
  static constexpr int value = (N1 == 5 && sizeof(R) == 8) ? 2 : 1;
};

template <int P, typename R, int MODE, int SCH>
__global__ __launch_bounds__((64 * (P + 1) * TilesPerGroup<P + 1, R>::value)) void stage_kernel(
    Geometry G, KTab<R, P + 1> T, StageArgs A) {
  constexpr int N1 = P + 1;
  constexpr int NSP = N1 * N1;
  constexpr int TPW = TilesPerGroup<N1, R>::value;
  constexpr bool LOB = SCH != kSchemeGlLp;      // Gauss-Lobatto points
  constexpr bool CHAIN = SCH == kSchemeGllChain;
  // float32 residuals are formed in deviation form (cpr_device.h)
  constexpr bool DEV = sizeof(R) == 4;
  constexpr int NT = 64 * N1;                   // lanes per tile
  constexpr int S = (NSP & 1) ? NSP : NSP + 1;  // odd LDS stride per element
  constexpr int VS = 64 * S;                    // LDS stride per variable
  __shared__ double qs_all[TPW][4 * VS];
  __shared__ R hF_all[TPW][4][kTile][N1][4];  // tile-boundary face fluxes: W, E, S, N

  if (A.skip != nullptr && *A.skip != 0) return;

  // tile of this group of waves; wave-uniform values live in scalar registers
  const int slot = TPW == 1 ? 0 : __builtin_amdgcn_readfirstlane((int)threadIdx.x / NT);
  const int tid = (int)threadIdx.x - slot * NT;
  const int lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int ntiles = G.ntx * G.nty;
  // groups of TPW tiles side by side in x: a grid of (ntx / TPW) x nty
  // groups when TPW divides ntx, else one run of groups in raster order
  const int tile = (G.ntx % TPW == 0 ? xcd_tile(blockIdx.x, G.ntx / TPW, G.nty)
                                     : xcd_tile(blockIdx.x, (ntiles + TPW - 1) / TPW, 1)) *
                       TPW + slot;
  const bool live = tile < ntiles;  // the last group's trailing slots may be empty
  const int tx = tile % G.ntx, ty = tile / G.ntx;
  const int I0 = tx * kTile, J0 = ty * kTile;
  const int nax = live ? min(kTile, G.nx - I0) : 0;
  const int nay = live ? min(kTile, G.ny - J0) : 0;
  const size_t plane = (size_t)G.ny * G.nx * NSP;
  const R gam = T.gam, gm1 = T.gm1;
  double* qs = qs_all[slot];
  auto hF = hF_all[slot];
  bool bad = false;

  using TC = TileCopy<N1, S>;
  const TC tc(lane);
  const int seg_len = nax * NSP;
  // paired copies where they pay: float64 from P = 2, float32 only with an
  // even number of points per element (its odd-P kernels lose occupancy to
  // the pair registers and run slower)
  constexpr bool PAIRS = TC::PAIRS && (sizeof(R) == 8 || NSP % 2 == 0);
  // paired copies need 16-byte aligned states (A.vec), even run offsets
  // (always when NSP is even; with NSP odd when nx is even, which makes
  // planes, rows and tile starts even) and whole pairs (seg_len even)
  const bool pairs_ok = A.vec && (NSP % 2 == 0 || (G.nx % 2 == 0 && seg_len % 2 == 0));

  // tile-boundary tasks: side hs (0 W, 1 E, 2 S, 3 N), position hp, line hm
  const bool halo = tid < 4 * kTile * N1;
  int hs = 0, hp = 0, hm = 0;
  bool hact = false, hout = false;
  R hq[4] = {R(0), R(0), R(0), R(0)};
  // deviation form: the neighbour's face state is formed in the frame of
  // the neighbour line's first point hr0 (the face point itself on
  // Gauss-Lobatto points) and moved into the own line's frame once that
  // line's reference is read from LDS
  double hr0[4] = {0.0, 0.0, 0.0, 0.0};

  // ---- A: tile -> LDS (coalesced along each tile row of elements) and the
  // outside neighbour lines, all loads issued before any is consumed ----
  {
    double v[TC::NRUN][TC::NIT];
    double2 v2[TC::NRUN][TC::NIT2];
#pragma unroll
    for (int u = 0; u < TC::NRUN; ++u) {
      const int sg = TC::run(wv, u);
      const int k = sg >> 3, cy = sg & 7;
      const bool ok = sg < 4 * kTile && cy < nay;
      const double* src = A.q_src + k * plane + ((size_t)(J0 + cy) * G.nx + I0) * NSP;
      if (PAIRS && pairs_ok) {
#pragma unroll
        for (int it = 0; it < TC::NIT2; ++it) {
          const int f = 2 * (it * 64 + lane);
          if (ok && f < seg_len) v2[u][it] = *reinterpret_cast<const double2*>(src + f);
        }
      } else {
#pragma unroll
        for (int it = 0; it < TC::NIT; ++it) {
          const int f = it * 64 + lane;
          if (ok && f < seg_len) v[u][it] = src[f];
        }
      }
    }
    // the outside neighbour lines of the tile-boundary lanes are scattered
    // loads. In float64 from P = 2 they are issued once the tile's coalesced
    // copies are written to LDS: a second round trip for those lanes, but the
    // copies no longer queue behind them and the copy registers are free
    // (P = 4 1024^2: 657 -> 605 us per launch; P = 2: 128 -> 95 VGPRs, five
    // waves per SIMD, the limited 512^2 step 233 -> 229 us). In float32 and
    // at P = 1 they go out with the copies (the later order measured 1-2 %
    // slower there).
    constexpr bool HALO_LATE = sizeof(R) == 8 && N1 >= 3;
    double hraw[4][N1];
    if constexpr (!HALO_LATE) {
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
          const double* base = A.q_src + ((size_t)Jo * G.nx + Io) * NSP;
          if (LOB) {
            // the neighbour's end point on the face that touches this tile
            const int nf = (hs == 0 || hs == 2) ? N1 - 1 : 0;
#pragma unroll
            for (int k = 0; k < 4; ++k)
              hraw[k][0] = base[k * plane + (hs < 2 ? hm * N1 + nf : nf * N1 + hm)];
          } else {
#pragma unroll
            for (int k = 0; k < 4; ++k)
#pragma unroll
              for (int n = 0; n < N1; ++n)
                hraw[k][n] = base[k * plane + (hs < 2 ? hm * N1 + n : n * N1 + hm)];
          }
        }
      }
    }
#pragma unroll
    for (int u = 0; u < TC::NRUN; ++u) {
      const int sg = TC::run(wv, u);
      const int k = sg >> 3, cy = sg & 7;
      const bool ok = sg < 4 * kTile && cy < nay;
      double* dst = qs + k * VS + cy * kTile * S;
      if (PAIRS && pairs_ok) {
#pragma unroll
        for (int it = 0; it < TC::NIT2; ++it) {
          const int f = 2 * (it * 64 + lane);
          if (ok && f < seg_len) {
            dst[tc.loff2[it]] = v2[u][it].x;
            dst[tc.loff2b[it]] = v2[u][it].y;
          }
        }
      } else {
#pragma unroll
        for (int it = 0; it < TC::NIT; ++it) {
          const int f = it * 64 + lane;
          if (ok && f < seg_len) dst[tc.loff[it]] = v[u][it];
        }
      }
    }
    if constexpr (HALO_LATE) {
      // the same task and loads as above, once the copies are in LDS
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
          const double* base = A.q_src + ((size_t)Jo * G.nx + Io) * NSP;
          if (LOB) {
            // the neighbour's end point on the face that touches this tile
            const int nf = (hs == 0 || hs == 2) ? N1 - 1 : 0;
#pragma unroll
            for (int k = 0; k < 4; ++k)
              hraw[k][0] = base[k * plane + (hs < 2 ? hm * N1 + nf : nf * N1 + hm)];
          } else {
#pragma unroll
            for (int k = 0; k < 4; ++k)
#pragma unroll
              for (int n = 0; n < N1; ++n)
                hraw[k][n] = base[k * plane + (hs < 2 ? hm * N1 + n : n * N1 + hm)];
          }
        }
      }
    }
    if (LOB && halo && hact && hout) {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        if (DEV)
          hr0[k] = hraw[k][0];
        else
          hq[k] = (R)hraw[k][0];
      }
    } else if (halo && hact && hout) {
      R ln[4][N1];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        if (DEV) hr0[k] = hraw[k][0];
        ln[k][0] = DEV ? R(0) : (R)hraw[k][0];
#pragma unroll
        for (int n = 1; n < N1; ++n) ln[k][n] = (R)(hraw[k][n] - hr0[k]);
      }
      // the neighbour's face that touches this tile
      const bool hi = (hs == 0 || hs == 2);
#pragma unroll
      for (int k = 0; k < 4; ++k)
        hq[k] = dot_n<N1>([&](int n) { return hi ? T.ep(n) : T.em(n); }, ln[k]);
    }
  }
  __syncthreads();

  // ---- B: tile-boundary fluxes; every lane reads its column ----
  if (halo && hact) {
    int e, stride, off;
    if (hs < 2) {  // row hm of element (0 or nax-1, hp)
      e = hp * kTile + (hs == 0 ? 0 : nax - 1);
      off = hm * N1;
      stride = 1;
    } else {  // column hm of element (hp, 0 or nay-1)
      e = (hs == 2 ? 0 : nay - 1) * kTile + hp;
      off = hm;
      stride = N1;
    }
    const bool lo = (hs == 0 || hs == 2);
    // own line's reference (deviation form): its first point
    double ref[4] = {0.0, 0.0, 0.0, 0.0};
    if (DEV) {
#pragma unroll
      for (int k = 0; k < 4; ++k) ref[k] = qs[k * VS + e * S + off];
    }
    R qin[4];
    if (LOB) {
      const int n = lo ? 0 : N1 - 1;
#pragma unroll
      for (int k = 0; k < 4; ++k) qin[k] = (R)(qs[k * VS + e * S + off + n * stride] - ref[k]);
    } else {
      R ln[4][N1];
#pragma unroll
      for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int n = 0; n < N1; ++n) ln[k][n] = (R)(qs[k * VS + e * S + off + n * stride] - ref[k]);
#pragma unroll
      for (int k = 0; k < 4; ++k)
        qin[k] = dot_n<N1>([&](int n) { return lo ? T.em(n) : T.ep(n); }, ln[k]);
    }
    if (!hout) {
#pragma unroll
      for (int k = 0; k < 4; ++k) hq[k] = qin[k];
    } else if (DEV) {
#pragma unroll
      for (int k = 0; k < 4; ++k) hq[k] = LOB ? (R)(hr0[k] - ref[k]) : (R)(hr0[k] - ref[k]) + hq[k];
    }
    const bool lo_side = (hs == 0 || hs == 2);  // neighbour is on the left/below
    R qL[4], qR[4], Fh[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      qL[k] = lo_side ? hq[k] : qin[k];
      qR[k] = lo_side ? qin[k] : hq[k];
    }
    if constexpr (DEV) {
      if (hs < 2)
        rusanov_dev<0>(qL, qR, dev_ref<0, R>(ref, gm1), gam, gm1, Fh, bad);
      else
        rusanov_dev<1>(qL, qR, dev_ref<1, R>(ref, gm1), gam, gm1, Fh, bad);
    } else {
      if (hs < 2)
        rusanov<0>(qL, qR, gam, gm1, Fh, bad);
      else
        rusanov<1>(qL, qR, gam, gm1, Fh, bad);
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) hF[hs][hp][hm][k] = Fh[k];
  }

  // both sweeps: lane -> element (cx = lane % 8, cy = lane / 8); row wv in
  // the x sweep (x neighbours 1 lane apart), column wv in the y sweep (y
  // neighbours 8 lanes apart). In both sweeps consecutive lanes read
  // consecutive elements of the odd-stride image, which spreads a wave's
  // LDS accesses over the banks.
  const int cxX = lane & 7, cyX = lane >> 3, eX = lane;
  const int cxY = lane & 7, cyY = lane >> 3, eY = lane;
  const bool actX = cxX < nax && cyX < nay;
  const bool actY = cxY < nax && cyY < nay;
  R qcol[4][N1];
  // deviation form: the column's reference (its first point), and the
  // differences to the references of the columns below and above, whose
  // face state and face flux enter this column's frame (lanes at the tile
  // edge read a clamped, unused element: their faces come from hF)
  double rc[4] = {0.0, 0.0, 0.0, 0.0};
  R dbel[4], dabv[4];
  if constexpr (DEV) {
    const int eb = eY >= kTile ? eY - kTile : eY, ea = eY < 64 - kTile ? eY + kTile : eY;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      rc[k] = qs[k * VS + eY * S + wv];
      dbel[k] = (R)(qs[k * VS + eb * S + wv] - rc[k]);
      dabv[k] = (R)(qs[k * VS + ea * S + wv] - rc[k]);
    }
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    qcol[k][0] = DEV ? R(0) : (R)qs[k * VS + eY * S + wv];
#pragma unroll
    for (int n = 1; n < N1; ++n) qcol[k][n] = (R)(qs[k * VS + eY * S + n * N1 + wv] - rc[k]);
  }
  __syncthreads();  // tile-boundary fluxes are in hF

  const double dt = (A.dt_dev != nullptr) ? *A.dt_dev : A.dt;

  // ---- C: column sweep ----
  R ry[4][N1];
  {
    R qlo[4], qhi[4], flo[4], fhi[4], dF[4][N1];
    bool b1 = false, b2 = false;
    R qnb[4], Fs[4], Fn[4];
    if constexpr (DEV) {
      const DevRef<R> c = dev_ref<1, R>(rc, gm1);
      if constexpr (CHAIN)
        line_ops_chain_dev<N1, 1>(qcol, c, T, gm1, qlo, qhi, flo, fhi, dF, b1);
      else
        line_ops_dev<N1, 1, LOB>(qcol, c, T, gm1, qlo, qhi, flo, fhi, dF, b1);
      // the element below: its face state moves into this frame by the
      // difference of the references; the face flux the element above forms
      // in its frame moves into this one by the flux deviation of theirs
#pragma unroll
      for (int k = 0; k < 4; ++k) qnb[k] = dbel[k] + __shfl_up(qhi[k], kTile, 64);
      rusanov_dev<1>(qnb, qlo, c, gam, gm1, Fs, b2);
      if (cyY == 0) {
#pragma unroll
        for (int k = 0; k < 4; ++k) Fs[k] = hF[2][cxY][wv][k];
        b2 = false;
      }
      R fa[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) Fn[k] = __shfl_down(Fs[k], kTile, 64);
      (void)dev_flux<1>(dabv, c, gm1, fa);
#pragma unroll
      for (int k = 0; k < 4; ++k) Fn[k] = Fn[k] + fa[k];
    } else {
      if constexpr (CHAIN)
        line_ops_chain<N1, 1>(qcol, T, gm1, qlo, qhi, flo, fhi, dF, b1);
      else
        line_ops<N1, 1, LOB>(qcol, T, gm1, qlo, qhi, flo, fhi, dF, b1);
#pragma unroll
      for (int k = 0; k < 4; ++k) qnb[k] = __shfl_up(qhi[k], kTile, 64);
      rusanov<1>(qnb, qlo, gam, gm1, Fs, b2);
      if (cyY == 0) {
#pragma unroll
        for (int k = 0; k < 4; ++k) Fs[k] = hF[2][cxY][wv][k];
        b2 = false;
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) Fn[k] = __shfl_down(Fs[k], kTile, 64);
    }
    if (cyY == nay - 1) {
#pragma unroll
      for (int k = 0; k < 4; ++k) Fn[k] = hF[3][cxY][wv][k];
    }
    const R rd = T.rdy;
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
      for (int n = 0; n < N1; ++n)
        ry[k][n] = rd * r_fma(Fn[k] - fhi[k], T.gR(n), r_fma(Fs[k] - flo[k], T.gL(n), dF[k][n]));
    if (actY) bad = bad || b1 || b2;
  }

  double qrow[4][N1];
#pragma unroll
  for (int k = 0; k < 4; ++k)
#pragma unroll
    for (int n = 0; n < N1; ++n) qrow[k][n] = qs[k * VS + eX * S + wv * N1 + n];
  // deviation form: differences of the west and east rows' references to
  // this row's (clamped, unused elements at the tile edge)
  R dwst[4], deas[4];
  if constexpr (DEV) {
    const int ew = eX > 0 ? eX - 1 : eX, ee = eX < 63 ? eX + 1 : eX;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      dwst[k] = (R)(qs[k * VS + ew * S + wv * N1] - qrow[k][0]);
      deas[k] = (R)(qs[k * VS + ee * S + wv * N1] - qrow[k][0]);
    }
  }
  __syncthreads();  // every row has been read
#pragma unroll
  for (int k = 0; k < 4; ++k)
#pragma unroll
    for (int n = 0; n < N1; ++n) qs[k * VS + eY * S + n * N1 + wv] = (double)ry[k][n];

  // ---- D: row sweep ----
  R rx[4][N1];
  {
    R qr[4][N1];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      // deviation form: the row's first point is its reference
      qr[k][0] = DEV ? R(0) : (R)qrow[k][0];
#pragma unroll
      for (int n = 1; n < N1; ++n) qr[k][n] = (R)(qrow[k][n] - (DEV ? qrow[k][0] : 0.0));
    }
    R qlo[4], qhi[4], flo[4], fhi[4], dF[4][N1];
    bool b1 = false, b2 = false;
    R qnb[4], Fw[4], Fe[4];
    if constexpr (DEV) {
      double rr[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) rr[k] = qrow[k][0];
      const DevRef<R> c = dev_ref<0, R>(rr, gm1);
      if constexpr (CHAIN)
        line_ops_chain_dev<N1, 0>(qr, c, T, gm1, qlo, qhi, flo, fhi, dF, b1);
      else
        line_ops_dev<N1, 0, LOB>(qr, c, T, gm1, qlo, qhi, flo, fhi, dF, b1);
#pragma unroll
      for (int k = 0; k < 4; ++k) qnb[k] = dwst[k] + __shfl_up(qhi[k], 1, 64);
      rusanov_dev<0>(qnb, qlo, c, gam, gm1, Fw, b2);
      if (cxX == 0) {
#pragma unroll
        for (int k = 0; k < 4; ++k) Fw[k] = hF[0][cyX][wv][k];
        b2 = false;
      }
      R fa[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) Fe[k] = __shfl_down(Fw[k], 1, 64);
      (void)dev_flux<0>(deas, c, gm1, fa);
#pragma unroll
      for (int k = 0; k < 4; ++k) Fe[k] = Fe[k] + fa[k];
    } else {
      if constexpr (CHAIN)
        line_ops_chain<N1, 0>(qr, T, gm1, qlo, qhi, flo, fhi, dF, b1);
      else
        line_ops<N1, 0, LOB>(qr, T, gm1, qlo, qhi, flo, fhi, dF, b1);
#pragma unroll
      for (int k = 0; k < 4; ++k) qnb[k] = __shfl_up(qhi[k], 1, 64);
      rusanov<0>(qnb, qlo, gam, gm1, Fw, b2);
      if (cxX == 0) {
#pragma unroll
        for (int k = 0; k < 4; ++k) Fw[k] = hF[0][cyX][wv][k];
        b2 = false;
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) Fe[k] = __shfl_down(Fw[k], 1, 64);
    }
    if (cxX == nax - 1) {
#pragma unroll
      for (int k = 0; k < 4; ++k) Fe[k] = hF[1][cyX][wv][k];
    }
    const R rd = T.rdx;
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
      for (int n = 0; n < N1; ++n)
        rx[k][n] = rd * r_fma(Fe[k] - fhi[k], T.gR(n), r_fma(Fw[k] - flo[k], T.gL(n), dF[k][n]));
    if (actX) bad = bad || b1 || b2;
  }

  __syncthreads();  // all column parts parked

#pragma unroll
  for (int k = 0; k < 4; ++k)
#pragma unroll
    for (int n = 0; n < N1; ++n) {
      const int a = k * VS + eX * S + wv * N1 + n;
      // explicit rounding: a fused rx + ry would round the two sweeps'
      // parts differently and break the x <-> y symmetry of the scheme
      const R rt = sym_add(rx[k][n], (R)qs[a]);
      if (MODE == kStageRK)
        qs[a] = A.b * fma(dt, (double)rt, qrow[k][n]);
      else
        qs[a] = (double)rt;
    }
  __syncthreads();

  // ---- E: coalesced epilogue ----
  // all of a wave's q_n loads are issued before its stores, which may
  // overwrite q_n in place
  const bool need_qn = MODE == kStageRK && A.a != 0.0;
  if (PAIRS && pairs_ok) {
    // the same in pairs of values (16-byte accesses)
    double2 vn[TC::NRUN][TC::NIT2];
#pragma unroll
    for (int u = 0; u < TC::NRUN; ++u) {
      const int sg = TC::run(wv, u);
      const int k = sg >> 3, cy = sg & 7;
      const bool ok = need_qn && sg < 4 * kTile && cy < nay;
      const double* src = A.q_n + k * plane + ((size_t)(J0 + cy) * G.nx + I0) * NSP;
#pragma unroll
      for (int it = 0; it < TC::NIT2; ++it) {
        const int f = 2 * (it * 64 + lane);
        if (ok && f < seg_len) vn[u][it] = *reinterpret_cast<const double2*>(src + f);
      }
    }
#pragma unroll
    for (int u = 0; u < TC::NRUN; ++u) {
      const int sg = TC::run(wv, u);
      const int cy = sg & 7, k = sg >> 3;
      const bool ok = sg < 4 * kTile && cy < nay;
      double* img = qs + k * VS + cy * kTile * S;
#pragma unroll
      for (int it = 0; it < TC::NIT2; ++it) {
        const int f = 2 * (it * 64 + lane);
        if (ok && f < seg_len) {
          const double a0 = img[tc.loff2[it]], a1 = img[tc.loff2b[it]];
          vn[u][it].x = need_qn ? fma(A.a, vn[u][it].x, a0) : a0;
          vn[u][it].y = need_qn ? fma(A.a, vn[u][it].y, a1) : a1;
          if (A.qbar != nullptr) {  // the output stays in LDS for its element means
            img[tc.loff2[it]] = vn[u][it].x;
            img[tc.loff2b[it]] = vn[u][it].y;
          }
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
        if (ok && f < seg_len) {
          if (MODE == kStageRK) {
            *reinterpret_cast<double2*>(A.q_dst + gb + f) = vn[u][it];
          } else {
            R* ro = static_cast<R*>(A.r_out) + gb + f;
            ro[0] = (R)vn[u][it].x;
            ro[1] = (R)vn[u][it].y;
          }
        }
      }
    }
  } else {
    double vn[TC::NRUN][TC::NIT];
#pragma unroll
    for (int u = 0; u < TC::NRUN; ++u) {
      const int sg = TC::run(wv, u);
      const int k = sg >> 3, cy = sg & 7;
      const bool ok = need_qn && sg < 4 * kTile && cy < nay;
      const double* src = A.q_n + k * plane + ((size_t)(J0 + cy) * G.nx + I0) * NSP;
#pragma unroll
      for (int it = 0; it < TC::NIT; ++it) {
        const int f = it * 64 + lane;
        if (ok && f < seg_len) vn[u][it] = src[f];
      }
    }
    // every output value of the wave is formed before the first store: a
    // store issued between two uses of loaded data would make the later use
    // wait for the store as well
#pragma unroll
    for (int u = 0; u < TC::NRUN; ++u) {
      const int sg = TC::run(wv, u);
      const int cy = sg & 7, k = sg >> 3;
      const bool ok = sg < 4 * kTile && cy < nay;
      double* img = qs + k * VS + cy * kTile * S;
#pragma unroll
      for (int it = 0; it < TC::NIT; ++it) {
        const int f = it * 64 + lane;
        if (ok && f < seg_len) {
          const double v = img[tc.loff[it]];
          vn[u][it] = need_qn ? fma(A.a, vn[u][it], v) : v;
          if (A.qbar != nullptr) img[tc.loff[it]] = vn[u][it];
        }
      }
    }
    // the loads above sit in lane-predicated blocks, after which the
    // compiler cannot tell that they have all returned and would wait for
    // every earlier store before each store; one explicit wait settles it
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
        if (ok && f < seg_len) {
          if (MODE == kStageRK)
            A.q_dst[gb + f] = vn[u][it];
          else
            static_cast<R*>(A.r_out)[gb + f] = (R)vn[u][it];
        }
      }
    }
  }

  // element means of the output for the limiter pass that follows: the
  // (i,j) and (j,i) terms are added as a pair first, in the same order as
  // the limiter's own means kernel, so the two give the same bits
  if (MODE == kStageRK && A.qbar != nullptr) {
    __syncthreads();
    const int ne = G.nx * G.ny;
    for (int t = tid; t < 4 * 64; t += NT) {
      const int k = t >> 6, e = t & 63, cx = e & 7, cy = e >> 3;
      if (cx < nax && cy < nay) {
        const double* v = qs + k * VS + e * S;
        double sm = 0.0;
#pragma unroll
        for (int j = 0; j < N1; ++j) {
          sm = fma(A.w[j] * A.w[j], v[j * N1 + j], sm);
#pragma unroll
          for (int i = j + 1; i < N1; ++i) sm = fma(A.w[i] * A.w[j], v[j * N1 + i] + v[i * N1 + j], sm);
        }
        A.qbar[k * ne + (J0 + cy) * G.nx + I0 + cx] = 0.25 * sm;
      }
    }
  }

  if (bad) atomicOr(A.err, 1);
}

template <int P, typename R, int SCH>
static hipError_t launch_stage_s(int mode, const Geometry& g, const KTab<R, P + 1>& kt,
                                 const StageArgs& a, hipStream_t s) {
  constexpr int TPW = TilesPerGroup<P + 1, R>::value;
  const dim3 grid((g.ntx * g.nty + TPW - 1) / TPW), block(64 * (P + 1) * TPW);
  if (mode == kStageRK)
    hipLaunchKernelGGL((stage_kernel<P, R, kStageRK, SCH>), grid, block, 0, s, g, kt, a);
  else
    hipLaunchKernelGGL((stage_kernel<P, R, kStageResidual, SCH>), grid, block, 0, s, g, kt, a);
  return hipGetLastError();
}

template <int P, typename R>
static hipError_t launch_stage_t(int scheme, int mode, const Geometry& g, const Tables1D& T,
                                 const StageArgs& a, hipStream_t s) {
  if (T.points != scheme_points(scheme)) return hipErrorInvalidValue;
  const KTab<R, P + 1> kt = make_ktab<R, P + 1>(T, g);
  switch (scheme) {
    case kSchemeGlLp: return launch_stage_s<P, R, kSchemeGlLp>(mode, g, kt, a, s);
    case kSchemeGllChain: return launch_stage_s<P, R, kSchemeGllChain>(mode, g, kt, a, s);
    case kSchemeGllLp: return launch_stage_s<P, R, kSchemeGllLp>(mode, g, kt, a, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_stage(int P, bool fp32, int scheme, int mode, const Geometry& g,
                        const Tables1D& T, const StageArgs& a, hipStream_t s) {
  switch (P) {
    case 1: return fp32 ? launch_stage_t<1, float>(scheme, mode, g, T, a, s) : launch_stage_t<1, double>(scheme, mode, g, T, a, s);
    case 2: return fp32 ? launch_stage_t<2, float>(scheme, mode, g, T, a, s) : launch_stage_t<2, double>(scheme, mode, g, T, a, s);
    case 3: return fp32 ? launch_stage_t<3, float>(scheme, mode, g, T, a, s) : launch_stage_t<3, double>(scheme, mode, g, T, a, s);
    case 4: return fp32 ? launch_stage_t<4, float>(scheme, mode, g, T, a, s) : launch_stage_t<4, double>(scheme, mode, g, T, a, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace cpr
