/*
 * cpr.h - C ABI of the MI355X CPR library for the 2D Euler equations.
 *
 * The library evaluates and advances the Correction Procedure via
 * Reconstruction (CPR) discretisation of the compressible Euler equations
 * on a uniform structured mesh of quadrilaterals (Zimmerman, Regele, Wie,
 * "A Comparative Study of 2D Numerical Methods with GPU Computing",
 * arXiv:1709.01619; Section 2 for the equations and the CPR differential
 * form, Section 2.6 for the slope limiter, Section 4 for the Rusanov flux,
 * the three-stage Runge-Kutta scheme and the CFL condition).
 *
 * Discretisation (scheme CPR_SCHEME_GL_LP, the default): P+1
 * Gauss-Legendre solution points per direction per element; face states
 * extrapolated from each element's solution polynomial; Rusanov common flux
 * at face points; Radau (DG-equivalent) correction lift; divergence of the
 * degree-P flux interpolant; SSP-RK3 in Shu-Osher form. This scheme is
 * exactly conservative.
 *
 * Scheme CPR_SCHEME_GLL_CHAIN is the paper's own CPR (Section 2.2, Fig. 1(b),
 * and the CPR flux kernel of Algorithms 7 and 8): P+1 Gauss-Lobatto
 * solution points, so the face states are the end values of each line; the
 * divergence is the chain rule A(q) dq/dx + B(q) dq/dy with dq/dx the
 * derivative of the solution polynomial; the same Rusanov flux and Radau
 * lift. The chain rule does not telescope, so this scheme conserves mass
 * exactly but momentum and energy only to truncation error.
 *
 * Scheme CPR_SCHEME_GLL_LP is the paper's nodal DG (Section 2.4: D f plus
 * the lift M^-1 M^A of the face-flux jumps, on Gauss-Lobatto points), which
 * is the differential form above with the derivative of the flux
 * interpolant on the Gauss-Lobatto points: the Radau derivatives at those
 * nodes are the lift columns of the exact mass matrix. Exactly
 * conservative.
 *
 * State layout (every q, r, v, lambda buffer): contiguous float64 (float32
 * for the FP32-bulk residual output) array q[k][J][I][j][i] of
 * 4 * ny * nx * (P+1)^2 values, C order:
 *   k in 0..3  conserved variable (rho, rho*u, rho*v, e),
 *   J in 0..ny-1 element row (y), I in 0..nx-1 element column (x),
 *   j in 0..P  eta index, i in 0..P xi index of the solution point.
 * Solution point (I,J,i,j) sits at x = x0 + (I + 1/2 + xi_i/2) dx,
 * y = y0 + (J + 1/2 + xi_j/2) dy with xi the ascending nodes of the
 * context's point set (Gauss-Legendre, or Gauss-Lobatto for
 * CPR_SCHEME_GLL_CHAIN and CPR_SCHEME_GLL_LP).
 *
 * Ownership: all array arguments are device pointers owned by the caller
 * (unless documented as host pointers). The library owns its scratch,
 * allocated in cpr_init and released in cpr_destroy; no other call
 * allocates device memory.
 *
 * Asynchrony: calls enqueue work on the context's HIP stream and return.
 * Argument errors return at once and enqueue nothing. A non-physical state
 * met inside a kernel (rho <= 0, p <= 0 or NaN) sets a device flag that the
 * next synchronising call (cpr_sync, and every call that returns a host
 * value) reports as CPR_ENONPHYSICAL and clears.
 *
 * Threading: a context is not thread-safe; separate contexts are
 * independent. Overlapping calls on one context must share its stream.
 */
#ifndef CPR_H
#define CPR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CPR_ABI_VERSION 2

typedef struct cpr_ctx cpr_ctx;

typedef enum {
  CPR_OK = 0,
  CPR_EINVAL = -1,         /* bad argument or configuration            */
  CPR_ENOMEM = -2,         /* device allocation failed                 */
  CPR_EHIP = -3,           /* HIP runtime error                        */
  CPR_EUNSUPPORTED = -4,   /* valid request this build does not serve  */
  CPR_ENONPHYSICAL = -5    /* rho <= 0, p <= 0 or NaN met on device    */
} cpr_status;

enum { CPR_BC_PERIODIC = 0, CPR_BC_TRANSMISSIVE = 1 };
enum { CPR_FP64 = 0, CPR_FP32_BULK = 1 };
enum { CPR_LIM_NONE = 0, CPR_LIM_TVB_CHAR = 1 };
enum { CPR_SCHEME_GL_LP = 0, CPR_SCHEME_GLL_CHAIN = 1, CPR_SCHEME_GLL_LP = 2 };

typedef struct {
  int32_t abi_version;  /* must equal CPR_ABI_VERSION                     */
  int32_t order_p;      /* polynomial degree P, 1..4                      */
  int32_t nx, ny;       /* elements per direction, 1..2^20 each, and
                           nx*ny <= 2^29                                  */
  double x0, x1;        /* domain [x0,x1] x [y0,y1], x1 > x0, y1 > y0     */
  double y0, y1;
  int32_t bc;           /* CPR_BC_PERIODIC or CPR_BC_TRANSMISSIVE         */
  int32_t precision;    /* CPR_FP64, or CPR_FP32_BULK: residual in float32
                           (accumulated in float32), state, RK update,
                           sums and norms in float64                     */
  double gamma;         /* ratio of specific heats, > 1                   */
  int32_t limiter;      /* CPR_LIM_NONE or CPR_LIM_TVB_CHAR               */
  int32_t scheme;       /* CPR_SCHEME_GL_LP, CPR_SCHEME_GLL_CHAIN or
                           CPR_SCHEME_GLL_LP                              */
  double tvb_m;         /* TVB constant M >= 0 (limiter only)             */
  double cfl;           /* CFL number for device-computed dt, > 0         */
  double t_end;         /* final time for device-computed dt (clips the
                           last step); <= 0 means no clipping            */
} cpr_config;

/* Create a context (Section 2.2 tables for degree P on the scheme's point
 * set, scratch for the RK
 * stages, the limiter and the adjoint). stream: a hipStream_t, or NULL for
 * the null stream. Returns CPR_EINVAL for an invalid configuration or NULL
 * cfg/out, CPR_ENOMEM if scratch cannot be allocated (nothing leaks). */
cpr_status cpr_init(const cpr_config* cfg, void* stream, cpr_ctx** out);

/* Release the context and its scratch. NULL is accepted. Waits for the
 * context's stream. */
cpr_status cpr_destroy(cpr_ctx* ctx);

/* Change the stream later calls enqueue on. */
cpr_status cpr_set_stream(cpr_ctx* ctx, void* stream);

/* r = R(q) = dq/dt of the CPR semi-discretisation (Section 2.2, the
 * differential form with the Radau correction; Rusanov face flux of
 * Section 4) in the context's scheme. q: device float64 state. r: device
 * buffer of the same shape, float64 (CPR_FP64) or float32 (CPR_FP32_BULK);
 * r must not alias q. */
cpr_status cpr_residual(cpr_ctx* ctx, const double* q, void* r);

/* Advance q (device, in place) by one SSP-RK3 step of size dt in Shu-Osher
 * form (Section 4, three-stage Runge-Kutta):
 *   q1 = qn + dt R(qn); q2 = 3/4 qn + 1/4 (q1 + dt R(q1));
 *   q(n+1) = 1/3 qn + 2/3 (q2 + dt R(q2)).
 * dt > 0: that step. dt <= 0: dt = min(cfl * h / max(|u|+c), t_end - t) is
 * computed on the device from qn (h = min(dx, dy); Section 4 CFL
 * condition) and the context's device time t advances; once t >= t_end the
 * call leaves q unchanged. apply_limiter != 0 applies the context's
 * limiter after each stage (Section 2.6); CPR_EUNSUPPORTED if the context
 * has CPR_LIM_NONE. */
cpr_status cpr_rk3_step(cpr_ctx* ctx, double* q, double dt, int32_t apply_limiter);

/* Apply the TVB characteristic minmod limiter to q (device, in place):
 * element means, face means of the extrapolated state, troubled-element
 * test on characteristic variables, linear reconstruction with limited
 * slopes in troubled elements (Section 2.6, eq. limu, in its TVB form).
 * flags: nullable device int32[ny*nx], set to 1 for troubled elements
 * else 0. n_troubled: nullable host pointer; when given, the call
 * synchronises and stores the number of troubled elements. */
cpr_status cpr_limit(cpr_ctx* ctx, double* q, int32_t* flags, int32_t* n_troubled);

/* out = (dR/dq)^T v at state q: the exact transpose of cpr_residual's
 * map, including the derivative of Rusanov's wave-speed bound
 * lam = max(|u_n|+c) over the two face states (derivative of |u_n| at 0 is
 * +1; where the two speeds tie to 1e-12 relative (2^-17 in CPR_FP32_BULK
 * contexts, above the float32 rounding of the speeds), the mean of the two
 * sides' gradients is used). In CPR_FP32_BULK contexts J^T v is evaluated
 * in float32 (as the residual is, from q and v rounded to float32) and
 * combined with v, x and y in float64. q, v, out: device float64 states;
 * out must not alias
 * q or v. For CPR_SCHEME_GLL_CHAIN the divergence A(q_i) (Dq)_i transposes
 * into sum_i D_il A(q_i)^T a_i plus the flux's second derivatives
 * d/dq [a_l . A(q) (Dq)_l] at q_l (a = -(2/h) v), evaluated together on
 * dual numbers q_l + eps (Dq)_l. */
cpr_status cpr_residual_vjp(cpr_ctx* ctx, const double* q, const double* v, double* out);

/* Discrete adjoint of one unlimited SSP-RK3 step of size dt > 0 from q_n:
 * lam_n = (d q(n+1) / d q_n)^T lam_np1, recomputing the stage states.
 *   lam2 = 2/3 (lam3 + dt J(q2)^T lam3); lam1 = 1/4 (lam2 + dt J(q1)^T lam2);
 *   lam_n = lam1 + dt J(qn)^T lam1 + 1/3 lam3 + 3/4 lam2.
 * All pointers device float64 states; lam_n may alias lam_np1. In
 * CPR_FP32_BULK contexts the stage states are recomputed with the float32
 * residual and the J^T products are float32 (cpr_residual_vjp); the lam
 * combinations are float64. CPR_EUNSUPPORTED on a context with a limiter. */
cpr_status cpr_adjoint_step(cpr_ctx* ctx, const double* q_n, double dt,
                            const double* lam_np1, double* lam_n);

/* One unlimited SSP-RK3 step of size dt > 0 from q_n (as cpr_rk3_step with
 * that dt and no limiter) that also hands back its stage states:
 * q1 = qn + dt R(qn), q2 = 3/4 qn + 1/4 (q1 + dt R(q1)), and
 * q_out = q(n+1) = 1/3 qn + 2/3 (q2 + dt R(q2)). q_out may be q_n (the step
 * in place); otherwise q_n is left unchanged. For adjoint sweeps that keep
 * the states of a checkpoint segment (cpr_adjoint_step_stages), which then
 * need not recompute them, and that chain the steps of the segment without
 * copies. All pointers device float64 states; q_n, q1 and q2 distinct, and
 * q_out distinct from q1 and q2 (CPR_EINVAL otherwise). */
cpr_status cpr_rk3_step_stages(cpr_ctx* ctx, double* q_n, double dt, double* q1, double* q2,
                               double* q_out);

/* cpr_adjoint_step with the step's stage states q1, q2 supplied (from
 * cpr_rk3_step_stages on q_n and the same dt) instead of recomputed: the
 * three transposes only, lam2 = 2/3 (lam3 + dt J(q2)^T lam3),
 * lam1 = 1/4 (lam2 + dt J(q1)^T lam2),
 * lam_n = lam1 + dt J(qn)^T lam1 + 1/3 lam3 + 3/4 lam2. Same results, bit for
 * bit, as cpr_adjoint_step. lam_n may alias lam_np1, not q_n, q1 or q2.
 * CPR_EUNSUPPORTED as cpr_adjoint_step. */
cpr_status cpr_adjoint_step_stages(cpr_ctx* ctx, const double* q_n, const double* q1,
                                   const double* q2, double dt, const double* lam_np1,
                                   double* lam_n);

/* Largest sqrt(u^2+v^2) + c over all solution points of q (device);
 * synchronises; result to *out_host. */
cpr_status cpr_max_wavespeed(cpr_ctx* ctx, const double* q, double* out_host);

/* Domain integrals of the four conserved variables by the tensor rule of
 * the context's point set, sum w_i w_j (dx dy / 4) q; synchronises;
 * out_host[4] (host). */
cpr_status cpr_integrals(cpr_ctx* ctx, const double* q, double* out_host);

/* Area-normalised quadrature L2 norm of a[var] - b[var]:
 * sqrt(sum w_i w_j (dx dy/4) (a-b)^2 / |domain|). a, b: device float64
 * states; b may be NULL (norm of a). var in 0..3. Synchronises. */
cpr_status cpr_l2_diff(cpr_ctx* ctx, const double* a, const double* b, int32_t var,
                       double* out_host);

/* Physical coordinates of every solution point, device float64 arrays x,
 * y of ny*nx*(P+1)^2 values each, layout [J][I][j][i]. */
cpr_status cpr_point_coords(cpr_ctx* ctx, double* x, double* y);

/* The library's 1D tables for degree P (host arrays of P+1 values, any may
 * be NULL): Gauss-Legendre nodes and weights, and the Radau correction
 * derivatives gL'(xi_i), gR'(xi_i). No context or device needed.
 * CPR_EINVAL for P outside 1..4. */
cpr_status cpr_tables(int32_t order_p, double* xi, double* w, double* gLp, double* gRp);

/* The same tables for a scheme's point set: CPR_SCHEME_GL_LP as
 * cpr_tables; CPR_SCHEME_GLL_CHAIN and CPR_SCHEME_GLL_LP the
 * Gauss-Lobatto-Legendre nodes (-1, the roots of L_P', +1), weights
 * 2 / (P (P+1) L_P(xi)^2), and the Radau correction derivatives at those
 * nodes (Section 2.2). No context or device
 * needed. CPR_EINVAL for an unknown scheme or P outside 1..4. */
cpr_status cpr_scheme_tables(int32_t scheme, int32_t order_p, double* xi, double* w, double* gLp,
                             double* gRp);

/* Device time of the CFL-driven stepping (cpr_rk3_step with dt <= 0). */
cpr_status cpr_set_time(cpr_ctx* ctx, double t);
cpr_status cpr_get_time(cpr_ctx* ctx, double* t_host, double* last_dt_host);

/* Number of troubled-element detections summed over every limiter pass of
 * the context (cpr_limit calls and the passes inside cpr_rk3_step) since
 * cpr_init or the last reset: the limiter activity of Section 2.6's
 * detection step, e.g. the troubled fraction of a run is
 * total / (passes x nx x ny). Synchronises; stores the count in
 * *total_host; reset != 0 clears the total after reading. */
cpr_status cpr_troubled_total(cpr_ctx* ctx, int64_t* total_host, int32_t reset);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): one
 * unlimited SSP-RK3 step of fixed size dt, as cpr_rk3_step(ctx, q, dt, 0)
 * on a context made from *cfg gives bit for bit, but without a context.
 * It allocates nothing: the two stage states live in a static device array
 * of the library, 2 x 32 MiB plus a few words, which every GPU the
 * library runs on holds until the process ends. The array's address is
 * looked up on the first call on each device (make that first call
 * outside graph capture).
 *   cfg     configuration as for cpr_init (host pointer, read during the
 *           call only); limiter must be CPR_LIM_NONE (CPR_EUNSUPPORTED
 *           otherwise).
 *   stream  hipStream_t the kernels are enqueued on, or NULL.
 *   q       device float64 state (layout above), advanced in place.
 *   dt      step size, finite and > 0 (no device-computed dt).
 *   err_flag nullable device int32 the kernels set to 1 on a non-physical
 *           state; the caller clears and reads it. NULL: the flag goes to
 *           a word of the static array, cleared by the call, and is lost.
 * Returns CPR_EINVAL for an invalid cfg, NULL q or bad dt, and
 * CPR_EUNSUPPORTED when the state exceeds 2^22 float64 values (32 MiB,
 * e.g. P = 3 on 256 x 256 elements); nothing is enqueued then, and
 * cpr_last_error(NULL) gives the reason. Asynchronous otherwise. Every
 * call on one GPU uses the same static array, so calls that overlap on one
 * GPU (several streams or host threads at once) race; serialise them. */
cpr_status cpr_rk3_step_static(const cpr_config* cfg, void* stream, double* q, double dt,
                               int32_t* err_flag);

/* Wait for the context's stream; return any deferred device error. */
cpr_status cpr_sync(cpr_ctx* ctx);

const char* cpr_status_string(cpr_status s);
/* Text of the context's last error (never NULL; "" when none). With ctx
 * NULL: the last error of a context-free call (cpr_rk3_step_static) on the
 * calling host thread. */
const char* cpr_last_error(const cpr_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* CPR_H */
