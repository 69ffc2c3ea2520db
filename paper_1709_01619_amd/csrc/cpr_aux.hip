// Limiter, reductions and helpers for the CPR library (gfx950).
//
// Limiter (Section 2.6 of arXiv:1709.01619, eq. limu, in the TVB
// characteristic form of Cockburn and Shu that the paper cites): a means
// pass writes every element's average; a second pass, two lanes per element
// (one per direction), forms the face means of the extrapolated state, tests
// the face deviations against the neighbour differences on characteristic
// variables with the TVB minmod, and rewrites troubled elements as
// qbar + (x-x_I) s_x + (y-y_J) s_y with characteristic minmod slopes.
#include "cpr_device.h"

namespace cpr {

template <int N1>
struct WTab {
  double w[N1];
  double xi[N1];
  double em[N1];
  double ep[N1];
};

template <int N1>
static WTab<N1> make_wtab(const Tables1D& T) {
  WTab<N1> t;
  for (int i = 0; i < N1; ++i) {
    t.w[i] = T.w[i];
    t.xi[i] = T.xi[i];
    t.em[i] = T.em[i];
    t.ep[i] = T.ep[i];
  }
  return t;
}

// ---------------------------------------------------------------- means --
template <int P>
__global__ __launch_bounds__(256) void means_kernel(Geometry G, WTab<P + 1> W, LimitArgs A) {
  constexpr int N1 = P + 1, NSP = N1 * N1;
  if (A.skip != nullptr && *A.skip != 0) return;
  const int ne = G.nx * G.ny;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ne) return;
  const size_t plane = (size_t)ne * NSP;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const double* q = A.q + k * plane + (size_t)e * NSP;
    // the (i,j) and (j,i) terms are added as a pair first, so that the mean
    // of a transposed element is bitwise the same
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < N1; ++j) {
      s = fma(W.w[j] * W.w[j], q[j * N1 + j], s);
#pragma unroll
      for (int i = j + 1; i < N1; ++i) s = fma(W.w[i] * W.w[j], q[j * N1 + i] + q[i * N1 + j], s);
    }
    A.qbar[k * ne + e] = 0.25 * s;
  }
}

// Right (R) and left (L = R^-1) eigenvectors of the flux Jacobian in
// direction n at state qb, in (rho, m_n, m_t, e) order, where m_n and m_t
// are the momenta normal and tangential to n. The x direction takes
// (m_n, m_t) = (rho u, rho v), the y direction (rho v, rho u). The rows are
// formed one at a time from these scalars where they are used, so that no
// 4x4 matrix is held in registers.
struct CharState {
  double u, v, ke, c, H, b1, b2;
};

__device__ __forceinline__ CharState char_state(const double qb[4], double gamma) {
  CharState s;
  const double rho = qb[0];
  s.u = qb[1] / rho;
  s.v = qb[2] / rho;
  s.ke = 0.5 * sym_dot2(s.u, s.u, s.v, s.v);
  const double p = (gamma - 1.0) * (qb[3] - rho * s.ke);
  s.c = sqrt(gamma * p / rho);
  s.H = (qb[3] + p) / rho;
  s.b1 = (gamma - 1.0) / (s.c * s.c);
  s.b2 = s.ke * s.b1;
  return s;
}

// Row a of L, as coefficients of (rho, m_n, m_t, e), for the velocity
// components un normal and ut tangential to the direction.
__device__ __forceinline__ void left_row(const CharState& s, double un, double ut, int a,
                                         double r[4]) {
  const double b1 = s.b1, b2 = s.b2, c = s.c;
  if (a == 0) {
    r[0] = 0.5 * (b2 + un / c); r[1] = -0.5 * (b1 * un + 1.0 / c);
    r[2] = -0.5 * b1 * ut;      r[3] = 0.5 * b1;
  }
  if (a == 1) { r[0] = 1.0 - b2; r[1] = b1 * un; r[2] = b1 * ut; r[3] = -b1; }
  if (a == 2) { r[0] = -ut; r[1] = 0.0; r[2] = 1.0; r[3] = 0.0; }
  if (a == 3) {
    r[0] = 0.5 * (b2 - un / c); r[1] = -0.5 * (b1 * un - 1.0 / c);
    r[2] = -0.5 * b1 * ut;      r[3] = 0.5 * b1;
  }
}

// Row a of R (component a of (rho, m_n, m_t, e)), as coefficients of the
// four characteristic variables.
__device__ __forceinline__ void right_row(const CharState& s, double un, double ut, int a,
                                          double r[4]) {
  const double c = s.c;
  if (a == 0) { r[0] = 1.0; r[1] = 1.0; r[2] = 0.0; r[3] = 1.0; }
  if (a == 1) { r[0] = un - c; r[1] = un; r[2] = 0.0; r[3] = un + c; }
  if (a == 2) { r[0] = ut; r[1] = ut; r[2] = 1.0; r[3] = ut; }
  if (a == 3) { r[0] = s.H - un * c; r[1] = s.ke; r[2] = ut; r[3] = s.H + un * c; }
}

// r . (x0, xn, xt, x3): the normal and tangential momentum terms are summed
// as a pair, so that the x and y directions of transposed data round
// identically.
__device__ __forceinline__ double row_dot(const double r[4], double x0, double xn, double xt,
                                          double x3) {
  return fma(r[0], x0, r[3] * x3) + sym_dot2(r[1], xn, r[2], xt);
}

__device__ __forceinline__ double minmod3(double a, double b, double c) {
  const bool pos = a > 0.0 && b > 0.0 && c > 0.0;
  const bool neg = a < 0.0 && b < 0.0 && c < 0.0;
  const double m = fmin(fmin(fabs(a), fabs(b)), fabs(c));
  return pos ? m : (neg ? -m : 0.0);
}

// ---------------------------------------------------- detect and limit --
// Each element has two adjacent lanes: the even one takes the x direction
// (west and east faces, extrapolated along rows), the odd one the y direction
// (south and north faces, along columns). A lane picks its direction by
// selects, not branches, so that both lanes of a pair run the same
// instructions, and it forms every quantity by the same operations as the
// direction alone would. limit_lane gives the element's mean qb, this
// direction's limited slope sl (components rho, rho u, rho v, e; d/dx on the
// x lane, d/dy on the y lane) and whether its TVB test finds the element
// troubled; false when the mean density is not positive.
template <int P>
__device__ __forceinline__ bool limit_lane(const Geometry& G, const WTab<P + 1>& W,
                                           const LimitArgs& A, int e, bool y, double qb[4],
                                           double sl[4], bool& troubled) {
  constexpr int N1 = P + 1, NSP = N1 * N1;
  const int I = e % G.nx, J = e / G.nx;
  const int ne = G.nx * G.ny;
  const size_t plane = (size_t)ne * NSP;
  // face means: each row (x) or column (y) extrapolated to its two ends,
  // weighted along the face and halved (faces have length 2 in reference
  // coordinates)
  double lo[4], hi[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    double v[NSP];
#pragma unroll
    for (int p = 0; p < NSP; ++p) v[p] = A.q[k * plane + (size_t)e * NSP + p];
    double l_ = 0.0, h_ = 0.0;
#pragma unroll
    for (int j = 0; j < N1; ++j) {
      double rl = 0.0, rh = 0.0;
#pragma unroll
      for (int i = 0; i < N1; ++i) {
        const double x = y ? v[i * N1 + j] : v[j * N1 + i];
        rl = fma(W.em[i], x, rl);
        rh = fma(W.ep[i], x, rh);
      }
      l_ = fma(W.w[j], rl, l_);
      h_ = fma(W.w[j], rh, h_);
    }
    lo[k] = 0.5 * l_;
    hi[k] = 0.5 * h_;
    qb[k] = A.qbar[k * ne + e];
  }
  troubled = false;
  if (!(qb[0] > 0.0)) return false;

  // neighbour elements on the low and high side (the element itself past a
  // transmissive boundary)
  int nl, nh;
  if (G.periodic) {
    nl = y ? ((J - 1 + G.ny) % G.ny) * G.nx + I : J * G.nx + (I - 1 + G.nx) % G.nx;
    nh = y ? ((J + 1) % G.ny) * G.nx + I : J * G.nx + (I + 1) % G.nx;
  } else {
    nl = y ? max(J - 1, 0) * G.nx + I : J * G.nx + max(I - 1, 0);
    nh = y ? min(J + 1, G.ny - 1) * G.nx + I : J * G.nx + min(I + 1, G.nx - 1);
  }
  double t0[4], t1[4], t2[4], t3[4], t4[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const double nlo = A.qbar[k * ne + nl], nhi = A.qbar[k * ne + nh];
    t0[k] = hi[k] - qb[k];
    t1[k] = qb[k] - lo[k];
    t2[k] = nhi - qb[k];
    t3[k] = qb[k] - nlo;
    t4[k] = hi[k] - lo[k];
  }
  const CharState s = char_state(qb, G.gamma);
  const double un = y ? s.v : s.u, ut = y ? s.u : s.v;
  const double h = y ? G.dy : G.dx;
  const double bound = A.tvb_m * h * h;
  // the normal and tangential momentum components of a difference
  const auto mn = [&](const double* t) { return y ? t[2] : t[1]; };
  const auto mt = [&](const double* t) { return y ? t[1] : t[2]; };
  double sc[4];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    double r[4];
    left_row(s, un, ut, a, r);
    const double up = row_dot(r, t0[0], mn(t0), mt(t0), t0[3]);
    const double um = row_dot(r, t1[0], mn(t1), mt(t1), t1[3]);
    const double dp = row_dot(r, t2[0], mn(t2), mt(t2), t2[3]);
    const double dm = row_dot(r, t3[0], mn(t3), mt(t3), t3[3]);
    const double dd = row_dot(r, t4[0], mn(t4), mt(t4), t4[3]);
    // the TVB-modified minmod leaves a deviation within bound unchanged and
    // otherwise replaces it by minmod(deviation, dp, dm); the element is
    // troubled when a deviation changes. Both minmods are formed and the
    // test is taken without branches.
    const double mp = minmod3(up, dp, dm);
    const double mm = minmod3(um, dp, dm);
    troubled = troubled | (!(fabs(up) <= bound) & (mp != up)) |
               (!(fabs(um) <= bound) & (mm != um));
    // minmod of the three differences over h, with one division: for h > 0
    // the rounded quotient is monotone in its numerator and keeps its sign,
    // so minmod(x/h, y/h, z/h) and minmod(x, y, z)/h are the same value (a
    // zero result can differ in sign only where a difference underflows
    // to zero on division, which needs h > 1)
    sc[a] = minmod3(dd, dp, dm) / h;
  }
  double sn = 0.0, st = 0.0;
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    double r[4];
    right_row(s, un, ut, a, r);
    const double o = row_dot(r, sc[0], sc[1], sc[2], sc[3]);
    if (a == 0) sl[0] = o;
    if (a == 1) sn = o;
    if (a == 2) st = o;
    if (a == 3) sl[3] = o;
  }
  sl[1] = y ? st : sn;  // rho u: normal on the x lane, tangential on the y lane
  sl[2] = y ? sn : st;
  return true;
}

// Detect and limit, two lanes per element (limit_lane). The pair combines its
// troubled flags and exchanges its slopes by lane shuffles; in a troubled
// element each lane rewrites two of the four variables as the mean plus the
// limited linear part.
template <int P>
__global__ __launch_bounds__(256) void limit_kernel(Geometry G, WTab<P + 1> W, LimitArgs A) {
  constexpr int N1 = P + 1, NSP = N1 * N1;
  if (A.skip != nullptr && *A.skip != 0) return;  // the same for every block
  __shared__ int wave_count[4];
  const int ne = G.nx * G.ny;
  const int tix = blockIdx.x * blockDim.x + threadIdx.x;
  const int e = tix >> 1, d = tix & 1;  // both lanes of a pair are past ne together
  const size_t plane = (size_t)ne * NSP;
  bool tr = false, ok = true;
  double qb[4] = {0.0, 0.0, 0.0, 0.0}, sl[4] = {0.0, 0.0, 0.0, 0.0};
  if (e < ne) ok = limit_lane<P>(G, W, A, e, d != 0, qb, sl, tr);
  const bool troubled = tr | (__shfl_xor((int)tr, 1) != 0);
  double so[4];  // the other lane's slope
#pragma unroll
  for (int k = 0; k < 4; ++k) so[k] = __shfl_xor(sl[k], 1);
  if (e < ne && d == 0) {
    if (!ok)
      atomicOr(A.err, 1);
    else if (A.flags != nullptr)
      A.flags[e] = troubled ? 1 : 0;
  }

  // the block's troubled elements, counted on their x lanes: one count per
  // wave, summed by one thread; the running total has a slot per block, so
  // no two blocks add to the same address (a thousand atomics on one
  // address serialise at the L2)
  const unsigned long long tw = __ballot(troubled && d == 0 && e < ne);
  if ((threadIdx.x & 63) == 0) wave_count[threadIdx.x >> 6] = __popcll(tw);
  __syncthreads();
  if (threadIdx.x == 0) {
    int n = 0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) n += wave_count[w];
    if (A.count != nullptr && n != 0) atomicAdd(A.count, n);
    if (A.total != nullptr) A.total[blockIdx.x] += (unsigned long long)n;
  }
  if (!troubled || e >= ne) return;
  // variables 0 and 1 on the x lane, 2 and 3 on the y lane; each takes its
  // x slope from the x lane and its y slope from the y lane
  const double hx = 0.5 * G.dx, hy = 0.5 * G.dy;
  const double qa = d ? qb[2] : qb[0], qc = d ? qb[3] : qb[1];
  const double sxa = d ? so[2] : sl[0], sya = d ? sl[2] : so[0];
  const double sxc = d ? so[3] : sl[1], syc = d ? sl[3] : so[1];
  double* pa = A.q + (size_t)(2 * d) * plane + (size_t)e * NSP;
  double* pc = pa + plane;
#pragma unroll
  for (int j = 0; j < N1; ++j)
#pragma unroll
    for (int i = 0; i < N1; ++i) {
      pa[j * N1 + i] = qa + sym_dot2(sxa, hx * W.xi[i], sya, hy * W.xi[j]);
      pc[j * N1 + i] = qc + sym_dot2(sxc, hx * W.xi[i], syc, hy * W.xi[j]);
    }
}

// two lanes per element, 128 elements per block of 256
int limit_blocks(const Geometry& g) { return (g.nx * g.ny + 127) / 128; }

template <int P>
static hipError_t launch_limit_t(const Geometry& g, const Tables1D& T, const LimitArgs& a,
                                 hipStream_t s) {
  const WTab<P + 1> w = make_wtab<P + 1>(T);
  const dim3 grid(limit_blocks(g)), block(256);
  if (!a.means_ready)  // one lane per element
    hipLaunchKernelGGL((means_kernel<P>), dim3((g.nx * g.ny + 255) / 256), block, 0, s, g, w, a);
  hipLaunchKernelGGL((limit_kernel<P>), grid, block, 0, s, g, w, a);
  return hipGetLastError();
}

hipError_t launch_limit(int P, const Geometry& g, const Tables1D& T, const LimitArgs& a,
                        hipStream_t s) {
  switch (P) {
    case 1: return launch_limit_t<1>(g, T, a, s);
    case 2: return launch_limit_t<2>(g, T, a, s);
    case 3: return launch_limit_t<3>(g, T, a, s);
    case 4: return launch_limit_t<4>(g, T, a, s);
    default: return hipErrorInvalidValue;
  }
}

// ---------------------------------------------------------- reductions --
constexpr int kRedBlock = 256;
constexpr int kRedMaxBlocks = 1024;

static int red_blocks(size_t npts) {
  size_t b = (npts + kRedBlock - 1) / kRedBlock;
  if (b > (size_t)kRedMaxBlocks) b = kRedMaxBlocks;
  if (b < 1) b = 1;
  return (int)b;
}

size_t reduce_partials_size(int, const Geometry&) { return (size_t)kRedMaxBlocks * 4 + 8; }

// Largest point wave speed |V| + c of each block's share of the points into
// part[blockIdx.x] (one plain store per block: a thousand atomics on one
// address would serialise at the L2), and the non-physical flag.
template <int P>
__global__ __launch_bounds__(kRedBlock) void wavespeed_kernel(Geometry G, const double* q,
                                                              double* part, int* err) {
  constexpr int NSP = (P + 1) * (P + 1);
  __shared__ double red[kRedBlock];
  const size_t npts = (size_t)G.nx * G.ny * NSP;
  double m = 0.0;
  bool bad = false;
  for (size_t g = blockIdx.x * (size_t)kRedBlock + threadIdx.x; g < npts;
       g += (size_t)gridDim.x * kRedBlock) {
    const double rho = q[g], mx = q[npts + g], my = q[2 * npts + g], en = q[3 * npts + g];
    const double u = mx / rho, v = my / rho;
    const double p = (G.gamma - 1.0) * (en - 0.5 * sym_dot2(mx, u, my, v));
    bad = bad || !(rho > 0.0) || !(p > 0.0);
    const double s = sqrt(sym_dot2(u, u, v, v)) + sqrt(G.gamma * p / rho);
    if (s > m) m = s;
  }
  red[threadIdx.x] = m;
  __syncthreads();
  for (int o = kRedBlock / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
  if (bad) atomicOr(err, 1);
}

int wavespeed_parts(int P, const Geometry& g) {
  return red_blocks((size_t)g.nx * g.ny * (P + 1) * (P + 1));
}

hipError_t launch_max_wavespeed(int P, const Geometry& g, const double* q, double* part, int* err,
                                hipStream_t s) {
  const dim3 grid(wavespeed_parts(P, g)), block(kRedBlock);
  switch (P) {
    case 1: hipLaunchKernelGGL((wavespeed_kernel<1>), grid, block, 0, s, g, q, part, err); break;
    case 2: hipLaunchKernelGGL((wavespeed_kernel<2>), grid, block, 0, s, g, q, part, err); break;
    case 3: hipLaunchKernelGGL((wavespeed_kernel<3>), grid, block, 0, s, g, q, part, err); break;
    case 4: hipLaunchKernelGGL((wavespeed_kernel<4>), grid, block, 0, s, g, q, part, err); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// the largest of part[0 .. n) (all >= 0), in one block of kRedBlock threads:
// each thread's loads go out together (one memory round trip for n up to
// 4 kRedBlock, where a plain strided loop waits on each load in turn), then
// the maximum is taken within each wave by shuffles and over the waves in
// LDS; the maximum is exact in any order
__device__ __forceinline__ double block_max_parts(const double* part, int n, double* red) {
  constexpr int U = 4;
  double m = 0.0;
  for (int i0 = threadIdx.x; i0 < n; i0 += U * kRedBlock) {
    double v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = i0 + u * kRedBlock;
      v[u] = i < n ? part[i] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) m = fmax(m, v[u]);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  double r = red[0];
#pragma unroll
  for (int w = 1; w < kRedBlock / 64; ++w) r = fmax(r, red[w]);
  return r;
}

// The step's dt from the largest wave speed lam and the time tn, by thread
// 0: dt = min(cfl h / lam, t_end - tn) and t += dt, or skip once t_end is
// reached (t_end > 0).
__device__ __forceinline__ void cfl_dt_store(double lam, double tn, double cfl, double h,
                                             double t_end, double* t, double* dt, int* skip) {
  if (t_end > 0.0 && t_end - tn <= 1e-14 * t_end) {
    *skip = 1;
    *dt = 0.0;
    return;
  }
  double d = cfl * h / lam;
  if (t_end > 0.0 && d > t_end - tn) d = t_end - tn;
  *dt = d;
  *t = tn + d;
  *skip = 0;
}

__global__ __launch_bounds__(kRedBlock) void cfl_dt_kernel(const double* part, int nparts, double cfl,
                                                           double h, double t_end, double* t,
                                                           double* dt, int* skip) {
  __shared__ double red[kRedBlock / 64];
  // read before the reduction's barrier, so that its latency overlaps the
  // partials' and no thread reads t after thread 0 writes it
  const double tn = *t;
  const double lam = block_max_parts(part, nparts, red);
  if (threadIdx.x == 0) cfl_dt_store(lam, tn, cfl, h, t_end, t, dt, skip);
}

hipError_t launch_cfl_dt(const double* part, int nparts, double cfl, double h, double t_end,
                         double* t, double* dt, int* skip, hipStream_t s) {
  hipLaunchKernelGGL(cfl_dt_kernel, dim3(1), dim3(kRedBlock), 0, s, part, nparts, cfl, h, t_end, t,
                     dt, skip);
  return hipGetLastError();
}

__global__ __launch_bounds__(kRedBlock) void max_parts_kernel(const double* part, int nparts,
                                                              double* out) {
  __shared__ double red[kRedBlock / 64];
  const double m = block_max_parts(part, nparts, red);
  if (threadIdx.x == 0) *out = m;
}

hipError_t launch_max_parts(const double* part, int nparts, double* out, hipStream_t s) {
  hipLaunchKernelGGL(max_parts_kernel, dim3(1), dim3(kRedBlock), 0, s, part, nparts, out);
  return hipGetLastError();
}

template <int P>
__global__ __launch_bounds__(kRedBlock) void wsum_kernel(Geometry G, WTab<P + 1> W, int mode,
                                                         const double* a, const double* b,
                                                         int var, double* partials) {
  constexpr int N1 = P + 1, NSP = N1 * N1;
  __shared__ double red[4][kRedBlock];
  const size_t npts = (size_t)G.nx * G.ny * NSP;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (size_t g = blockIdx.x * (size_t)kRedBlock + threadIdx.x; g < npts;
       g += (size_t)gridDim.x * kRedBlock) {
    const int p = (int)(g % NSP);
    const double w = W.w[p / N1] * W.w[p % N1];
    if (mode == 0) {
#pragma unroll
      for (int k = 0; k < 4; ++k) acc[k] += w * a[k * npts + g];
    } else {
      const double d = a[var * npts + g] - (b != nullptr ? b[var * npts + g] : 0.0);
      acc[0] += w * d * d;
    }
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) red[k][threadIdx.x] = acc[k];
  __syncthreads();
  for (int o = kRedBlock / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
#pragma unroll
      for (int k = 0; k < 4; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x < 4) partials[blockIdx.x * 4 + threadIdx.x] = red[threadIdx.x][0];
}

__global__ __launch_bounds__(kRedBlock) void wsum_final_kernel(const double* partials, int nblocks,
                                                               int mode, double scale, double area,
                                                               double* out) {
  __shared__ double red[4][kRedBlock];
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int b = threadIdx.x; b < nblocks; b += kRedBlock)
#pragma unroll
    for (int k = 0; k < 4; ++k) acc[k] += partials[b * 4 + k];
#pragma unroll
  for (int k = 0; k < 4; ++k) red[k][threadIdx.x] = acc[k];
  __syncthreads();
  for (int o = kRedBlock / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
#pragma unroll
      for (int k = 0; k < 4; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    if (mode == 0) {
      for (int k = 0; k < 4; ++k) out[k] = scale * red[k][0];
    } else {
      out[0] = sqrt(scale * red[0][0] / area);
    }
  }
}

hipError_t launch_weighted_sum(int P, const Geometry& g, const Tables1D& T, int mode,
                               const double* a, const double* b, int var, double area,
                               double* partials, double* out, hipStream_t s) {
  const size_t npts = (size_t)g.nx * g.ny * (P + 1) * (P + 1);
  const int nb = red_blocks(npts);
  const dim3 grid(nb), block(kRedBlock);
  switch (P) {
    case 1: hipLaunchKernelGGL((wsum_kernel<1>), grid, block, 0, s, g, make_wtab<2>(T), mode, a, b, var, partials); break;
    case 2: hipLaunchKernelGGL((wsum_kernel<2>), grid, block, 0, s, g, make_wtab<3>(T), mode, a, b, var, partials); break;
    case 3: hipLaunchKernelGGL((wsum_kernel<3>), grid, block, 0, s, g, make_wtab<4>(T), mode, a, b, var, partials); break;
    case 4: hipLaunchKernelGGL((wsum_kernel<4>), grid, block, 0, s, g, make_wtab<5>(T), mode, a, b, var, partials); break;
    default: return hipErrorInvalidValue;
  }
  const double scale = 0.25 * g.dx * g.dy;
  hipLaunchKernelGGL(wsum_final_kernel, dim3(1), dim3(kRedBlock), 0, s, partials, nb, mode, scale,
                     area, out);
  return hipGetLastError();
}

// -------------------------------------------------------------- helpers --
template <int P>
__global__ __launch_bounds__(256) void coords_kernel(Geometry G, WTab<P + 1> W, double x0,
                                                     double y0, double* x, double* y) {
  constexpr int N1 = P + 1, NSP = N1 * N1;
  const size_t npts = (size_t)G.nx * G.ny * NSP;
  const size_t g = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (g >= npts) return;
  const size_t e = g / NSP;
  const int p = (int)(g - e * NSP);
  const int I = (int)(e % G.nx), J = (int)(e / G.nx);
  x[g] = x0 + (I + 0.5) * G.dx + 0.5 * G.dx * W.xi[p % N1];
  y[g] = y0 + (J + 0.5) * G.dy + 0.5 * G.dy * W.xi[p / N1];
}

hipError_t launch_coords(int P, const Geometry& g, const Tables1D& T, double x0, double y0,
                         double* x, double* y, hipStream_t s) {
  const size_t npts = (size_t)g.nx * g.ny * (P + 1) * (P + 1);
  const dim3 grid((unsigned)((npts + 255) / 256)), block(256);
  switch (P) {
    case 1: hipLaunchKernelGGL((coords_kernel<1>), grid, block, 0, s, g, make_wtab<2>(T), x0, y0, x, y); break;
    case 2: hipLaunchKernelGGL((coords_kernel<2>), grid, block, 0, s, g, make_wtab<3>(T), x0, y0, x, y); break;
    case 3: hipLaunchKernelGGL((coords_kernel<3>), grid, block, 0, s, g, make_wtab<4>(T), x0, y0, x, y); break;
    case 4: hipLaunchKernelGGL((coords_kernel<4>), grid, block, 0, s, g, make_wtab<5>(T), x0, y0, x, y); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

__global__ void fill_int_kernel(int* p, int v, size_t n) {
  const size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

hipError_t launch_fill_int(int* p, int v, size_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(fill_int_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}

}  // namespace cpr
