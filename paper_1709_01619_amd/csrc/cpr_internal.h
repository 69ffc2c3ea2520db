// Internal declarations shared by the host API and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "cpr.h"

namespace cpr {

constexpr int kMaxP = 4;
constexpr int kTile = 8;  // elements per tile edge; one tile per workgroup

// Solution point sets: Gauss-Legendre, or Gauss-Lobatto-Legendre (end
// points included).
enum { kGauss = 0, kLobatto = 1 };

// Discretisations (the values of cpr_config.scheme): Gauss-Legendre points
// with the derivative of the flux interpolant; Gauss-Lobatto points with the
// chain-rule divergence (the paper's CPR); Gauss-Lobatto points with the
// derivative of the flux interpolant (the paper's NDG).
enum { kSchemeGlLp = 0, kSchemeGllChain = 1, kSchemeGllLp = 2 };
inline int scheme_points(int scheme) { return scheme == kSchemeGlLp ? kGauss : kLobatto; }

// 1D tables on [-1, 1] for degree P, float64 (host).
struct Tables1D {
  int P;
  int points;                      // kGauss or kLobatto
  double xi[kMaxP + 1];
  double w[kMaxP + 1];
  double D[kMaxP + 1][kMaxP + 1];  // D[i][l] = l_l'(xi_i)
  double em[kMaxP + 1];            // l_l(-1)
  double ep[kMaxP + 1];            // l_l(+1)
  double gLp[kMaxP + 1];           // gL'(xi_i)
  double gRp[kMaxP + 1];           // gR'(xi_i)
};

bool build_tables(int P, int points, Tables1D* T);

struct Geometry {
  int nx, ny;    // elements
  int ntx, nty;  // tiles
  double dx, dy;
  double gamma;
  int periodic;
};

// One fused SSP-RK3 stage (mode kStageRK):
//   q_dst = a * q_n + b * (q_src + dt * R(q_src))   (q_n unused when a == 0)
// or the residual alone (mode kStageResidual): r_out = R(q_src).
struct StageArgs {
  const double* q_src;
  const double* q_n;
  double* q_dst;
  void* r_out;
  double a, b, dt;
  const double* dt_dev;  // when non-null, dt is read from here
  const int* skip;       // when non-null and *skip != 0, the kernel does nothing
  int* err;              // set to 1 on a non-physical state
  int vec;               // every state pointer is 16-byte aligned
  double* qbar;          // when non-null (RK mode): element means of q_dst, 4 * ny * nx
  double w[kMaxP + 1];   // quadrature weights for those means
};

enum { kStageRK = 0, kStageResidual = 1 };

hipError_t launch_stage(int P, bool fp32, int scheme, int mode, const Geometry& g,
                        const Tables1D& T, const StageArgs& a, hipStream_t s);

// out = alpha v + delta J(q)^T v + beta x + gam y   (x, y nullable), with
// J = dR/dq the Jacobian of the float64 residual.
struct VjpArgs {
  const double* q;
  const double* v;
  const double* x;
  const double* y;
  double* out;
  double alpha, delta, beta, gam;
  int* err;
  int vec;  // every state pointer is 16-byte aligned
};
hipError_t launch_vjp(int P, bool fp32, int scheme, const Geometry& g, const Tables1D& T,
                      const VjpArgs& a, hipStream_t s);

// Limiter: element means then detect + limit in place.
struct LimitArgs {
  double* q;
  double* qbar;     // 4 * ny * nx scratch
  int* flags;       // nullable, ny * nx
  int* count;       // nullable device counter of troubled elements (atomic add per block)
  unsigned long long* total;  // nullable running total of troubled elements, one slot
                              // per block of the limiter's grid (limit_blocks slots)
  double tvb_m;
  const int* skip;  // nullable
  int* err;
  int means_ready;  // qbar already holds the means of q (written by the stage kernel)
};
hipError_t launch_limit(int P, const Geometry& g, const Tables1D& T, const LimitArgs& a,
                        hipStream_t s);
// blocks of the limiter's grid
int limit_blocks(const Geometry& g);

// Reductions. partials must hold reduce_partials_size() doubles.
size_t reduce_partials_size(int P, const Geometry& g);
// The largest point wave speed |V| + c in two steps: launch_max_wavespeed
// writes one maximum per block into part[0 .. wavespeed_parts(P, g)) (part
// must hold that many doubles; reduce_partials_size() is enough), then
// launch_cfl_dt or launch_max_parts takes their maximum.
int wavespeed_parts(int P, const Geometry& g);
hipError_t launch_max_wavespeed(int P, const Geometry& g, const double* q, double* part, int* err,
                                hipStream_t s);
// lam = max(part[0 .. nparts)); dt = min(cfl h / lam, t_end - t); t += dt;
// skip when t >= t_end (t_end > 0).
hipError_t launch_cfl_dt(const double* part, int nparts, double cfl, double h, double t_end,
                         double* t, double* dt, int* skip, hipStream_t s);
// *out = max(part[0 .. nparts))
hipError_t launch_max_parts(const double* part, int nparts, double* out, hipStream_t s);
// Weighted sums: mode 0 -> out[0..3] = sum w_i w_j (dxdy/4) q_k;
// mode 1 -> out[0] = sqrt(sum w w (dxdy/4) (a-b)^2 / area) for variable var.
hipError_t launch_weighted_sum(int P, const Geometry& g, const Tables1D& T, int mode,
                               const double* a, const double* b, int var, double area,
                               double* partials, double* out, hipStream_t s);
hipError_t launch_coords(int P, const Geometry& g, const Tables1D& T, double x0, double y0,
                         double* x, double* y, hipStream_t s);
hipError_t launch_fill_int(int* p, int v, size_t n, hipStream_t s);

// Host helpers of the C ABI (cpr_api.hip).
bool config_valid(const cpr_config& c);
Geometry config_geometry(const cpr_config& c);
// Arguments of stage `stage` (0, 1, 2) of one unlimited SSP-RK3 step of
// fixed size dt from q: reads src (and q for stages 1, 2), writes dst.
void rk3_stage_args(const Tables1D& T, int P, int stage, const double* q, const double* src,
                    double* dst, double dt, int* err, StageArgs* s);
// Error text of context-free calls, per host thread (cpr_last_error(NULL)).
void set_thread_error(const char* fmt, ...);

}  // namespace cpr
