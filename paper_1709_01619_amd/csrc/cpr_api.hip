// C ABI of the CPR library: argument checking, context and scratch
// management, and the launch sequences of each entry point.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <vector>
#include <new>

#include "cpr.h"
#include "cpr_internal.h"

using namespace cpr;

static_assert(CPR_SCHEME_GL_LP == kSchemeGlLp && CPR_SCHEME_GLL_CHAIN == kSchemeGllChain &&
                  CPR_SCHEME_GLL_LP == kSchemeGllLp,
              "public and internal scheme values differ");

struct cpr_ctx {
  cpr_config cfg;
  Geometry geo;
  Tables1D tab;
  hipStream_t stream;
  int device;
  size_t n_state;  // float64 values per state
  size_t n_elem;
  double* q1;      // RK stage 1 state / adjoint recompute
  double* q2;      // RK stage 2 state / adjoint recompute
  double* lam1;    // adjoint stage cotangents
  double* lam2;
  double* qbar;    // element means (limiter)
  int* iscr;       // [0] error flag, [1] skip flag, [2] troubled count
  double* dscal;   // [0] t, [1] dt
  unsigned long long* troubled_total;  // running total, one slot per limiter block
  int n_total;                         // its slots
  double* partials;  // per-block partial sums and wave-speed maxima
  double* red_out;   // 4 doubles
  char last_error[512];
};

namespace cpr {

thread_local char t_last_error[256];

void set_thread_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(t_last_error, sizeof(t_last_error), fmt, ap);
  va_end(ap);
}

bool config_valid(const cpr_config& c) {
  if (c.abi_version != CPR_ABI_VERSION) return false;
  if (c.order_p < 1 || c.order_p > kMaxP) return false;
  if (c.nx < 1 || c.ny < 1 || c.nx > (1 << 20) || c.ny > (1 << 20)) return false;
  // element means are indexed k*nx*ny + e in 32-bit arithmetic
  if ((int64_t)c.nx * c.ny > ((int64_t)1 << 29)) return false;
  if (!(std::isfinite(c.x0) && std::isfinite(c.x1) && c.x1 > c.x0)) return false;
  if (!(std::isfinite(c.y0) && std::isfinite(c.y1) && c.y1 > c.y0)) return false;
  if (c.bc != CPR_BC_PERIODIC && c.bc != CPR_BC_TRANSMISSIVE) return false;
  if (c.precision != CPR_FP64 && c.precision != CPR_FP32_BULK) return false;
  if (!(std::isfinite(c.gamma) && c.gamma > 1.0)) return false;
  if (c.limiter != CPR_LIM_NONE && c.limiter != CPR_LIM_TVB_CHAR) return false;
  if (c.scheme != CPR_SCHEME_GL_LP && c.scheme != CPR_SCHEME_GLL_CHAIN &&
      c.scheme != CPR_SCHEME_GLL_LP)
    return false;
  if (!(std::isfinite(c.tvb_m) && c.tvb_m >= 0.0)) return false;
  if (!(std::isfinite(c.cfl) && c.cfl >= 0.0)) return false;
  if (!std::isfinite(c.t_end)) return false;
  return true;
}

Geometry config_geometry(const cpr_config& c) {
  Geometry g{};
  g.nx = c.nx;
  g.ny = c.ny;
  g.ntx = (c.nx + kTile - 1) / kTile;
  g.nty = (c.ny + kTile - 1) / kTile;
  g.dx = (c.x1 - c.x0) / c.nx;
  g.dy = (c.y1 - c.y0) / c.ny;
  g.gamma = c.gamma;
  g.periodic = c.bc == CPR_BC_PERIODIC ? 1 : 0;
  return g;
}

void rk3_stage_args(const Tables1D& T, int P, int stage, const double* q, const double* src,
                    double* dst, double dt, int* err, StageArgs* s) {
  static const double ka[3] = {0.0, 0.75, 1.0 / 3.0}, kb[3] = {1.0, 0.25, 2.0 / 3.0};
  *s = StageArgs{};
  for (int i = 0; i <= P; ++i) s->w[i] = T.w[i];
  s->q_src = src;
  s->q_n = stage == 0 ? nullptr : q;
  s->q_dst = dst;
  s->a = ka[stage];
  s->b = kb[stage];
  s->dt = dt;
  s->err = err;
  const uintptr_t any = (uintptr_t)src | (uintptr_t)q | (uintptr_t)dst;
  s->vec = (any & 15) == 0;
}

}  // namespace cpr

namespace {

void set_err(cpr_ctx* c, const char* fmt, ...) {
  if (c == nullptr) return;
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(c->last_error, sizeof(c->last_error), fmt, ap);
  va_end(ap);
}

cpr_status hip_fail(cpr_ctx* c, hipError_t e, const char* what) {
  set_err(c, "%s: %s", what, hipGetErrorString(e));
  return e == hipErrorOutOfMemory ? CPR_ENOMEM : CPR_EHIP;
}

#define HIP_TRY(ctx, expr, what)                     \
  do {                                               \
    hipError_t _e = (expr);                          \
    if (_e != hipSuccess) return hip_fail(ctx, _e, what); \
  } while (0)

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

void free_all(cpr_ctx* c) {
  double* bufs[] = {c->q1, c->q2, c->lam1, c->lam2, c->qbar, c->dscal, c->partials, c->red_out};
  for (double* b : bufs)
    if (b) (void)hipFree(b);
  if (c->iscr) (void)hipFree(c->iscr);
  if (c->troubled_total) (void)hipFree(c->troubled_total);
}

// Read back the deferred device error flag (synchronising) and clear it.
cpr_status check_device_error(cpr_ctx* c) {
  int flag = 0;
  HIP_TRY(c, hipMemcpyAsync(&flag, c->iscr, sizeof(int), hipMemcpyDeviceToHost, c->stream),
          "copy error flag");
  HIP_TRY(c, hipStreamSynchronize(c->stream), "stream synchronize");
  if (flag != 0) {
    HIP_TRY(c, launch_fill_int(c->iscr, 0, 1, c->stream), "clear error flag");
    set_err(c, "non-physical state (rho <= 0, p <= 0 or NaN) met on the device");
    return CPR_ENONPHYSICAL;
  }
  return CPR_OK;
}

cpr_status stage(cpr_ctx* c, int mode, const double* src, const double* qn, double* dst,
                 void* rout, double a, double b, double dt, bool device_dt, bool means = false) {
  StageArgs s{};
  s.qbar = means ? c->qbar : nullptr;
  for (int i = 0; i <= c->cfg.order_p; ++i) s.w[i] = c->tab.w[i];
  s.q_src = src;
  s.q_n = qn;
  s.q_dst = dst;
  s.r_out = rout;
  s.a = a;
  s.b = b;
  s.dt = dt;
  s.dt_dev = device_dt ? c->dscal + 1 : nullptr;
  s.skip = device_dt ? c->iscr + 1 : nullptr;
  s.err = c->iscr;
  const uintptr_t any = (uintptr_t)src | (uintptr_t)qn | (uintptr_t)dst | (uintptr_t)rout;
  s.vec = (any & 15) == 0;
  HIP_TRY(c, launch_stage(c->cfg.order_p, c->cfg.precision == CPR_FP32_BULK, c->cfg.scheme, mode,
                          c->geo, c->tab, s, c->stream),
          "stage kernel launch");
  return CPR_OK;
}

cpr_status limit_pass(cpr_ctx* c, double* q, int* flags, int* count, bool device_dt,
                      bool means_ready = false) {
  LimitArgs l{};
  l.means_ready = means_ready ? 1 : 0;
  l.q = q;
  l.qbar = c->qbar;
  l.flags = flags;
  l.count = count;
  l.total = c->troubled_total;
  l.tvb_m = c->cfg.tvb_m;
  l.skip = device_dt ? c->iscr + 1 : nullptr;
  l.err = c->iscr;
  HIP_TRY(c, launch_limit(c->cfg.order_p, c->geo, c->tab, l, c->stream), "limiter launch");
  return CPR_OK;
}

cpr_status vjp(cpr_ctx* c, const double* q, const double* v, const double* x, const double* y,
               double* out, double alpha, double delta, double beta, double gam) {
  VjpArgs a{};
  a.q = q;
  a.v = v;
  a.x = x;
  a.y = y;
  a.out = out;
  a.alpha = alpha;
  a.delta = delta;
  a.beta = beta;
  a.gam = gam;
  a.err = c->iscr;
  const uintptr_t any = (uintptr_t)q | (uintptr_t)v | (uintptr_t)x | (uintptr_t)y | (uintptr_t)out;
  a.vec = (any & 15) == 0;
  HIP_TRY(c, launch_vjp(c->cfg.order_p, c->cfg.precision == CPR_FP32_BULK, c->cfg.scheme, c->geo,
                        c->tab, a, c->stream),
          "adjoint kernel launch");
  return CPR_OK;
}

}  // namespace

extern "C" {

const char* cpr_status_string(cpr_status s) {
  switch (s) {
    case CPR_OK: return "ok";
    case CPR_EINVAL: return "invalid argument";
    case CPR_ENOMEM: return "out of device memory";
    case CPR_EHIP: return "HIP runtime error";
    case CPR_EUNSUPPORTED: return "unsupported";
    case CPR_ENONPHYSICAL: return "non-physical state";
    default: return "unknown status";
  }
}

const char* cpr_last_error(const cpr_ctx* ctx) { return ctx ? ctx->last_error : t_last_error; }

cpr_status cpr_tables(int32_t order_p, double* xi, double* w, double* gLp, double* gRp) {
  return cpr_scheme_tables(CPR_SCHEME_GL_LP, order_p, xi, w, gLp, gRp);
}

cpr_status cpr_scheme_tables(int32_t scheme, int32_t order_p, double* xi, double* w, double* gLp,
                             double* gRp) {
  if (scheme != CPR_SCHEME_GL_LP && scheme != CPR_SCHEME_GLL_CHAIN && scheme != CPR_SCHEME_GLL_LP)
    return CPR_EINVAL;
  Tables1D T;
  if (!build_tables(order_p, scheme_points(scheme), &T)) return CPR_EINVAL;
  for (int i = 0; i <= order_p; ++i) {
    if (xi) xi[i] = T.xi[i];
    if (w) w[i] = T.w[i];
    if (gLp) gLp[i] = T.gLp[i];
    if (gRp) gRp[i] = T.gRp[i];
  }
  return CPR_OK;
}

cpr_status cpr_init(const cpr_config* cfg, void* stream, cpr_ctx** out) {
  if (out == nullptr || cfg == nullptr) return CPR_EINVAL;
  *out = nullptr;
  const cpr_config& c = *cfg;
  if (!config_valid(c)) return CPR_EINVAL;

  cpr_ctx* x = new (std::nothrow) cpr_ctx();
  if (x == nullptr) return CPR_ENOMEM;
  std::memset(x, 0, sizeof(*x));
  x->cfg = c;
  x->stream = static_cast<hipStream_t>(stream);
  if (!build_tables(c.order_p, scheme_points(c.scheme), &x->tab)) {
    delete x;
    return CPR_EINVAL;
  }
  const int n1 = c.order_p + 1;
  x->geo = config_geometry(c);
  x->n_elem = (size_t)c.nx * (size_t)c.ny;
  x->n_state = 4 * x->n_elem * (size_t)(n1 * n1);
  if ((size_t)x->geo.ntx * (size_t)x->geo.nty >= (size_t)1 << 31) {
    delete x;
    return CPR_ENOMEM;
  }
  (void)hipGetDevice(&x->device);

  const size_t sb = x->n_state * sizeof(double);
  hipError_t e = hipSuccess;
  double** states[] = {&x->q1, &x->q2, &x->lam1, &x->lam2};
  for (double** p : states)
    if (e == hipSuccess) e = hipMalloc(p, sb);
  if (e == hipSuccess) e = hipMalloc(&x->qbar, 4 * x->n_elem * sizeof(double));
  if (e == hipSuccess) e = hipMalloc(&x->iscr, 10 * sizeof(int));
  if (e == hipSuccess) e = hipMalloc(&x->dscal, 4 * sizeof(double));
  if (e == hipSuccess) e = hipMalloc(&x->partials, reduce_partials_size(c.order_p, x->geo) * sizeof(double));
  if (e == hipSuccess) e = hipMalloc(&x->red_out, 4 * sizeof(double));
  x->n_total = limit_blocks(x->geo);
  if (e == hipSuccess) e = hipMalloc(&x->troubled_total, (size_t)x->n_total * sizeof(unsigned long long));
  if (e == hipSuccess)
    e = hipMemsetAsync(x->troubled_total, 0, (size_t)x->n_total * sizeof(unsigned long long), x->stream);
  if (e == hipSuccess) e = hipMemsetAsync(x->iscr, 0, 10 * sizeof(int), x->stream);
  if (e == hipSuccess) e = hipMemsetAsync(x->dscal, 0, 4 * sizeof(double), x->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(x->stream);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    free_all(x);
    const cpr_status st = e == hipErrorOutOfMemory ? CPR_ENOMEM : CPR_EHIP;
    delete x;
    return st;
  }
  *out = x;
  return CPR_OK;
}

cpr_status cpr_destroy(cpr_ctx* ctx) {
  if (ctx == nullptr) return CPR_OK;
  (void)hipStreamSynchronize(ctx->stream);
  free_all(ctx);
  delete ctx;
  return CPR_OK;
}

cpr_status cpr_set_stream(cpr_ctx* ctx, void* stream) {
  if (ctx == nullptr) return CPR_EINVAL;
  ctx->stream = static_cast<hipStream_t>(stream);
  return CPR_OK;
}

cpr_status cpr_residual(cpr_ctx* ctx, const double* q, void* r) {
  if (ctx == nullptr || q == nullptr || r == nullptr) return CPR_EINVAL;
  if ((const void*)q == r) {
    set_err(ctx, "cpr_residual: r must not alias q");
    return CPR_EINVAL;
  }
  return stage(ctx, kStageResidual, q, nullptr, nullptr, r, 0.0, 0.0, 0.0, false);
}

cpr_status cpr_rk3_step(cpr_ctx* ctx, double* q, double dt, int32_t apply_limiter) {
  if (ctx == nullptr || q == nullptr || !std::isfinite(dt)) return CPR_EINVAL;
  if (apply_limiter && ctx->cfg.limiter == CPR_LIM_NONE) {
    set_err(ctx, "cpr_rk3_step: the context has no limiter");
    return CPR_EUNSUPPORTED;
  }
  const bool ddt = dt <= 0.0;
  if (ddt) {
    if (!(ctx->cfg.cfl > 0.0)) {
      set_err(ctx, "cpr_rk3_step: device dt needs cfl > 0");
      return CPR_EINVAL;
    }
    const double h = ctx->geo.dx < ctx->geo.dy ? ctx->geo.dx : ctx->geo.dy;
    HIP_TRY(ctx, launch_max_wavespeed(ctx->cfg.order_p, ctx->geo, q, ctx->partials, ctx->iscr,
                                      ctx->stream), "wave speed launch");
    HIP_TRY(ctx, launch_cfl_dt(ctx->partials, wavespeed_parts(ctx->cfg.order_p, ctx->geo),
                               ctx->cfg.cfl, h, ctx->cfg.t_end, ctx->dscal, ctx->dscal + 1,
                               ctx->iscr + 1, ctx->stream), "dt launch");
  }
  cpr_status st;
  const bool lim = apply_limiter != 0;
  // with the limiter, each stage kernel also writes the element means of its
  // output, which the limiter pass after it then uses
  if ((st = stage(ctx, kStageRK, q, nullptr, ctx->q1, nullptr, 0.0, 1.0, dt, ddt, lim)) != CPR_OK) return st;
  if (lim && (st = limit_pass(ctx, ctx->q1, nullptr, nullptr, ddt, true)) != CPR_OK) return st;
  if ((st = stage(ctx, kStageRK, ctx->q1, q, ctx->q2, nullptr, 0.75, 0.25, dt, ddt, lim)) != CPR_OK) return st;
  if (lim && (st = limit_pass(ctx, ctx->q2, nullptr, nullptr, ddt, true)) != CPR_OK) return st;
  if ((st = stage(ctx, kStageRK, ctx->q2, q, q, nullptr, 1.0 / 3.0, 2.0 / 3.0, dt, ddt, lim)) != CPR_OK) return st;
  if (lim && (st = limit_pass(ctx, q, nullptr, nullptr, ddt, true)) != CPR_OK) return st;
  return CPR_OK;
}

cpr_status cpr_limit(cpr_ctx* ctx, double* q, int32_t* flags, int32_t* n_troubled) {
  if (ctx == nullptr || q == nullptr) return CPR_EINVAL;
  if (n_troubled != nullptr)
    HIP_TRY(ctx, launch_fill_int(ctx->iscr + 2, 0, 1, ctx->stream), "clear counter");
  cpr_status st = limit_pass(ctx, q, flags, n_troubled ? ctx->iscr + 2 : nullptr, false);
  if (st != CPR_OK) return st;
  if (n_troubled != nullptr) {
    int cnt = 0;
    HIP_TRY(ctx, hipMemcpyAsync(&cnt, ctx->iscr + 2, sizeof(int), hipMemcpyDeviceToHost, ctx->stream),
            "copy count");
    st = check_device_error(ctx);
    *n_troubled = cnt;
    return st;
  }
  return CPR_OK;
}

cpr_status cpr_residual_vjp(cpr_ctx* ctx, const double* q, const double* v, double* out) {
  if (ctx == nullptr || q == nullptr || v == nullptr || out == nullptr) return CPR_EINVAL;
  if (out == q || out == v) {
    set_err(ctx, "cpr_residual_vjp: out must not alias q or v");
    return CPR_EINVAL;
  }
  return vjp(ctx, q, v, nullptr, nullptr, out, 0.0, 1.0, 0.0, 0.0);
}

namespace {

// static: inside the extern "C" block the unnamed namespace alone leaves
// these helpers among the library's exported symbols
static cpr_status adjoint_checks(cpr_ctx* ctx, const char* who) {
  if (ctx->cfg.limiter != CPR_LIM_NONE) {
    set_err(ctx, "%s: the limiter is not differentiated", who);
    return CPR_EUNSUPPORTED;
  }
  return CPR_OK;
}

// The three transposes of one SSP-RK3 step, given its stage states.
static cpr_status adjoint_sweep(cpr_ctx* ctx, const double* q_n, const double* q1,
                                const double* q2, double dt, const double* lam_np1,
                                double* lam_n) {
  cpr_status st;
  // lam2 = 2/3 (lam3 + dt J(q2)^T lam3)
  if ((st = vjp(ctx, q2, lam_np1, nullptr, nullptr, ctx->lam2, 2.0 / 3.0, 2.0 / 3.0 * dt, 0.0, 0.0)) != CPR_OK) return st;
  // lam1 = 1/4 (lam2 + dt J(q1)^T lam2)
  if ((st = vjp(ctx, q1, ctx->lam2, nullptr, nullptr, ctx->lam1, 0.25, 0.25 * dt, 0.0, 0.0)) != CPR_OK) return st;
  // lam_n = lam1 + dt J(qn)^T lam1 + 1/3 lam3 + 3/4 lam2
  return vjp(ctx, q_n, ctx->lam1, lam_np1, ctx->lam2, lam_n, 1.0, dt, 1.0 / 3.0, 0.75);
}

}  // namespace

cpr_status cpr_adjoint_step(cpr_ctx* ctx, const double* q_n, double dt, const double* lam_np1,
                            double* lam_n) {
  if (ctx == nullptr || q_n == nullptr || lam_np1 == nullptr || lam_n == nullptr) return CPR_EINVAL;
  if (!(std::isfinite(dt) && dt > 0.0)) return CPR_EINVAL;
  cpr_status st = adjoint_checks(ctx, "cpr_adjoint_step");
  if (st != CPR_OK) return st;
  if ((const double*)lam_n == q_n) return CPR_EINVAL;
  // recompute the stage states q1, q2 from q_n
  if ((st = stage(ctx, kStageRK, q_n, nullptr, ctx->q1, nullptr, 0.0, 1.0, dt, false)) != CPR_OK) return st;
  if ((st = stage(ctx, kStageRK, ctx->q1, q_n, ctx->q2, nullptr, 0.75, 0.25, dt, false)) != CPR_OK) return st;
  return adjoint_sweep(ctx, q_n, ctx->q1, ctx->q2, dt, lam_np1, lam_n);
}

cpr_status cpr_rk3_step_stages(cpr_ctx* ctx, double* q_n, double dt, double* q1, double* q2,
                               double* q_out) {
  if (ctx == nullptr || q_n == nullptr || q1 == nullptr || q2 == nullptr || q_out == nullptr)
    return CPR_EINVAL;
  if (!(std::isfinite(dt) && dt > 0.0)) return CPR_EINVAL;
  if (q1 == q_n || q2 == q_n || q1 == q2 || q_out == q1 || q_out == q2) {
    set_err(ctx, "cpr_rk3_step_stages: q_n, q1 and q2 must be distinct, q_out must not be q1 or q2");
    return CPR_EINVAL;
  }
  cpr_status st;
  if ((st = stage(ctx, kStageRK, q_n, nullptr, q1, nullptr, 0.0, 1.0, dt, false)) != CPR_OK) return st;
  if ((st = stage(ctx, kStageRK, q1, q_n, q2, nullptr, 0.75, 0.25, dt, false)) != CPR_OK) return st;
  // out of place the third stage reads q2 and q_n and writes q_out, which
  // aliases neither (a tile may only overwrite what no other tile reads)
  return stage(ctx, kStageRK, q2, q_n, q_out, nullptr, 1.0 / 3.0, 2.0 / 3.0, dt, false);
}

cpr_status cpr_adjoint_step_stages(cpr_ctx* ctx, const double* q_n, const double* q1,
                                   const double* q2, double dt, const double* lam_np1,
                                   double* lam_n) {
  if (ctx == nullptr || q_n == nullptr || q1 == nullptr || q2 == nullptr || lam_np1 == nullptr ||
      lam_n == nullptr)
    return CPR_EINVAL;
  if (!(std::isfinite(dt) && dt > 0.0)) return CPR_EINVAL;
  cpr_status st = adjoint_checks(ctx, "cpr_adjoint_step_stages");
  if (st != CPR_OK) return st;
  if ((const double*)lam_n == q_n || (const double*)lam_n == q1 || (const double*)lam_n == q2) {
    set_err(ctx, "cpr_adjoint_step_stages: lam_n must not alias q_n, q1 or q2");
    return CPR_EINVAL;
  }
  return adjoint_sweep(ctx, q_n, q1, q2, dt, lam_np1, lam_n);
}

cpr_status cpr_max_wavespeed(cpr_ctx* ctx, const double* q, double* out_host) {
  if (ctx == nullptr || q == nullptr || out_host == nullptr) return CPR_EINVAL;
  HIP_TRY(ctx, launch_max_wavespeed(ctx->cfg.order_p, ctx->geo, q, ctx->partials, ctx->iscr,
                                    ctx->stream),
          "wave speed launch");
  HIP_TRY(ctx, launch_max_parts(ctx->partials, wavespeed_parts(ctx->cfg.order_p, ctx->geo),
                                ctx->red_out, ctx->stream),
          "wave speed maximum launch");
  double v = 0.0;
  HIP_TRY(ctx, hipMemcpyAsync(&v, ctx->red_out, sizeof(v), hipMemcpyDeviceToHost, ctx->stream),
          "copy max");
  cpr_status st = check_device_error(ctx);
  *out_host = v;
  return st;
}

cpr_status cpr_integrals(cpr_ctx* ctx, const double* q, double* out_host) {
  if (ctx == nullptr || q == nullptr || out_host == nullptr) return CPR_EINVAL;
  HIP_TRY(ctx, launch_weighted_sum(ctx->cfg.order_p, ctx->geo, ctx->tab, 0, q, nullptr, 0, 1.0,
                                   ctx->partials, ctx->red_out, ctx->stream), "integral launch");
  HIP_TRY(ctx, hipMemcpyAsync(out_host, ctx->red_out, 4 * sizeof(double), hipMemcpyDeviceToHost,
                              ctx->stream), "copy integrals");
  return check_device_error(ctx);
}

cpr_status cpr_l2_diff(cpr_ctx* ctx, const double* a, const double* b, int32_t var, double* out_host) {
  if (ctx == nullptr || a == nullptr || out_host == nullptr || var < 0 || var > 3) return CPR_EINVAL;
  const double area = (ctx->cfg.x1 - ctx->cfg.x0) * (ctx->cfg.y1 - ctx->cfg.y0);
  HIP_TRY(ctx, launch_weighted_sum(ctx->cfg.order_p, ctx->geo, ctx->tab, 1, a, b, var, area,
                                   ctx->partials, ctx->red_out, ctx->stream), "l2 launch");
  HIP_TRY(ctx, hipMemcpyAsync(out_host, ctx->red_out, sizeof(double), hipMemcpyDeviceToHost,
                              ctx->stream), "copy l2");
  return check_device_error(ctx);
}

cpr_status cpr_point_coords(cpr_ctx* ctx, double* x, double* y) {
  if (ctx == nullptr || x == nullptr || y == nullptr) return CPR_EINVAL;
  HIP_TRY(ctx, launch_coords(ctx->cfg.order_p, ctx->geo, ctx->tab, ctx->cfg.x0, ctx->cfg.y0, x, y,
                             ctx->stream), "coords launch");
  return CPR_OK;
}

cpr_status cpr_set_time(cpr_ctx* ctx, double t) {
  if (ctx == nullptr || !std::isfinite(t)) return CPR_EINVAL;
  HIP_TRY(ctx, hipMemcpyAsync(ctx->dscal, &t, sizeof(double), hipMemcpyHostToDevice, ctx->stream),
          "set time");
  HIP_TRY(ctx, launch_fill_int(ctx->iscr + 1, 0, 1, ctx->stream), "clear skip");
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream), "stream synchronize");
  return CPR_OK;
}

cpr_status cpr_get_time(cpr_ctx* ctx, double* t_host, double* last_dt_host) {
  if (ctx == nullptr) return CPR_EINVAL;
  double v[2] = {0.0, 0.0};
  HIP_TRY(ctx, hipMemcpyAsync(v, ctx->dscal, 2 * sizeof(double), hipMemcpyDeviceToHost, ctx->stream),
          "get time");
  cpr_status st = check_device_error(ctx);
  if (t_host) *t_host = v[0];
  if (last_dt_host) *last_dt_host = v[1];
  return st;
}

cpr_status cpr_troubled_total(cpr_ctx* ctx, int64_t* total_host, int32_t reset) {
  if (ctx == nullptr || total_host == nullptr) return CPR_EINVAL;
  std::vector<unsigned long long> v((size_t)ctx->n_total);
  HIP_TRY(ctx, hipMemcpyAsync(v.data(), ctx->troubled_total, v.size() * sizeof(unsigned long long),
                              hipMemcpyDeviceToHost, ctx->stream),
          "read troubled total");
  if (reset)
    HIP_TRY(ctx, launch_fill_int(reinterpret_cast<int*>(ctx->troubled_total), 0, 2 * v.size(), ctx->stream),
            "clear troubled total");
  cpr_status st = check_device_error(ctx);
  unsigned long long sum = 0;
  for (unsigned long long b : v) sum += b;
  *total_host = (int64_t)sum;
  return st;
}

cpr_status cpr_sync(cpr_ctx* ctx) {
  if (ctx == nullptr) return CPR_EINVAL;
  return check_device_error(ctx);
}

}  // extern "C"
