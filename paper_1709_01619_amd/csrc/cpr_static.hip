// cpr_rk3_step_static: one unlimited SSP-RK3 step without a context and
// without any device allocation, for callers that cannot allocate (code
// under HIP graph capture, tight serving loops, harnesses that forbid
// hipMalloc). The two stage states live in one file-scope device array of
// fixed size; every GPU the library runs on holds its own copy of it until
// the process ends.
//
// In host code the array's name is only a stand-in for the symbol: its
// device address on the current GPU is looked up once per device with
// hipGetSymbolAddress, and only that address is ever handed to a kernel.
#include <atomic>
#include <cmath>
#include <mutex>

#include "cpr.h"
#include "cpr_internal.h"

namespace {

using namespace cpr;

// Largest state (float64 values) the static scratch serves: 2^22 values,
// 32 MiB, e.g. P = 3 on 256 x 256 elements.
constexpr size_t kStaticStateMax = size_t(1) << 22;
// layout: stage state 1, stage state 2, then 32 words for the error flag
constexpr size_t kStaticWords = 2 * kStaticStateMax + 32;

__device__ __align__(256) double scratch[kStaticWords];

constexpr int kMaxDevices = 64;
std::atomic<double*> g_scratch[kMaxDevices];
std::mutex g_scratch_mu;

// Device address of `scratch` on device dev (current), resolved once.
hipError_t scratch_ptr(int dev, double** out) {
  double* p = g_scratch[dev].load(std::memory_order_acquire);
  if (p == nullptr) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    p = g_scratch[dev].load(std::memory_order_relaxed);
    if (p == nullptr) {
      void* a = nullptr;
      const hipError_t e = hipGetSymbolAddress(&a, HIP_SYMBOL(scratch));
      if (e != hipSuccess) return e;
      if (a == nullptr) return hipErrorInvalidSymbol;
      p = static_cast<double*>(a);
      g_scratch[dev].store(p, std::memory_order_release);
    }
  }
  *out = p;
  return hipSuccess;
}

cpr_status hip_status(hipError_t e, const char* what) {
  set_thread_error("cpr_rk3_step_static: %s: %s", what, hipGetErrorString(e));
  return e == hipErrorOutOfMemory ? CPR_ENOMEM : CPR_EHIP;
}

}  // namespace

extern "C" cpr_status cpr_rk3_step_static(const cpr_config* cfg, void* stream, double* q,
                                          double dt, int32_t* err_flag) {
  if (cfg == nullptr || q == nullptr || !config_valid(*cfg)) {
    set_thread_error("cpr_rk3_step_static: invalid configuration or NULL argument");
    return CPR_EINVAL;
  }
  if (!(std::isfinite(dt) && dt > 0.0)) {
    set_thread_error("cpr_rk3_step_static: dt must be finite and > 0");
    return CPR_EINVAL;
  }
  const cpr_config& c = *cfg;
  if (c.limiter != CPR_LIM_NONE) {
    set_thread_error("cpr_rk3_step_static: the limiter is not served (static scratch)");
    return CPR_EUNSUPPORTED;
  }
  const size_t n1 = (size_t)c.order_p + 1;
  const size_t n_state = 4 * (size_t)c.nx * (size_t)c.ny * n1 * n1;
  if (n_state > kStaticStateMax) {
    set_thread_error(
        "cpr_rk3_step_static: state of %zu values exceeds the static scratch limit of %zu "
        "values (32 MiB per state)",
        n_state, kStaticStateMax);
    return CPR_EUNSUPPORTED;
  }
  Tables1D T;
  if (!build_tables(c.order_p, scheme_points(c.scheme), &T)) {
    set_thread_error("cpr_rk3_step_static: no tables for this degree");
    return CPR_EINVAL;
  }
  const Geometry g = config_geometry(c);

  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_status(e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) {
    set_thread_error("cpr_rk3_step_static: device index %d beyond %d", dev, kMaxDevices);
    return CPR_EUNSUPPORTED;
  }
  double* base = nullptr;
  if ((e = scratch_ptr(dev, &base)) != hipSuccess) return hip_status(e, "hipGetSymbolAddress");
  double* s1 = base;
  double* s2 = base + kStaticStateMax;
  int* err = err_flag;
  const hipStream_t st = static_cast<hipStream_t>(stream);
  if (err == nullptr) {
    // the flag word is shared by every call on this GPU and keeps the last
    // call's value: clear it (a kernel, not a memset, so that the call can
    // be recorded into a graph)
    err = reinterpret_cast<int*>(base + 2 * kStaticStateMax);
    if ((e = launch_fill_int(err, 0, 1, st)) != hipSuccess) return hip_status(e, "clear flag");
  }
  const bool fp32 = c.precision == CPR_FP32_BULK;
  const double* src[3] = {q, s1, s2};
  double* dst[3] = {s1, s2, q};
  for (int k = 0; k < 3; ++k) {
    StageArgs a;
    rk3_stage_args(T, c.order_p, k, q, src[k], dst[k], dt, err, &a);
    if ((e = launch_stage(c.order_p, fp32, c.scheme, kStageRK, g, T, a, st)) != hipSuccess)
      return hip_status(e, "stage kernel launch");
  }
  return CPR_OK;
}
