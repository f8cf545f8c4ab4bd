// Host-side helpers shared by the 1-D and 2-D runtimes (runtime.hip,
// runtime2d.hip): the per-thread error string behind cs_last_error, launch
// status checks, a device fill, optional per-launch timing with hipEvents
// and the reduction of objective-trace partial sums.
#pragma once
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "cscirc.h"

namespace cs {
namespace rt {

extern thread_local std::string g_err;
cs_status fail(cs_status st, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
inline cs_status ok() {
  g_err.clear();
  return CS_OK;
}

#define CS_HIP(call)                                                                 \
  do {                                                                               \
    hipError_t e_ = (call);                                                          \
    if (e_ != hipSuccess)                                                            \
      return ::cs::rt::fail(CS_EHIP, "%s failed: %s", #call, hipGetErrorString(e_)); \
  } while (0)

#define CS_LAUNCH(call)                                                              \
  do {                                                                               \
    hipError_t e_ = (call);                                                          \
    if (e_ != hipSuccess)                                                            \
      return ::cs::rt::fail(CS_EHIP, "kernel launch failed: %s", hipGetErrorString(e_)); \
  } while (0)

// Guards the plan caches of both runtimes.
extern std::mutex g_mu;

int ilog2(int64_t v);
bool is_pow2(int64_t v);

// exp(-2 pi i e / L) in double precision, rounded to float.
float2 root(int64_t e, int64_t L);

// p[0 .. count) = v on stream s (a kernel, so it can be graph-captured).
cs_status fill(float* p, size_t count, float v, hipStream_t s);

// obj[t] = inv_2m * sum_i res[t][i] + lambda * sum_i l1[t][i], t < iters,
// each sum in double in a fixed order.
cs_status objective_reduce(const double* res, int nres, const double* l1, int nl1, double inv_2m,
                           double lambda, float* obj, int iters, hipStream_t s);

// out[0] = max(out[0], max_i |t[i]|^2); out[0] must start >= 0.
cs_status max_abs2(const float2* t, int count, float* out, hipStream_t s);

// Error flags of the batched solves' plans on device `dev`: read, cleared,
// reported as CS_EHIP if one was set (runtime_batch.hip).
cs_status batch_check_flags(int dev);

// Timed launch kinds (names as reported by cs_timing_read).
enum TimedKind {
  T_A_ISTA = 0, T_B_ISTA, T_A_ADMM, T_B_ADMM, T_S_ISTA, T_S_ADMM, T_BATCH,
  T_C2_ISTA, T_R2_ISTA, T_C2_ADMM, T_R2_ADMM, T_DIRECT, T_DIRECT_T, T_CP_ROW, T_CP_COL, T_COUNT
};
bool timing_on();
// Records the start (tok == -1 on entry) or the stop event of a launch.
hipError_t timed_mark(int kind, hipStream_t s, long* tok);

template <class F>
hipError_t timed(int kind, hipStream_t s, F&& launch) {
  if (!timing_on()) return launch();
  long tok = -1;
  hipError_t e = timed_mark(kind, s, &tok);
  if (e != hipSuccess) return e;
  e = launch();
  if (e != hipSuccess) return e;
  return timed_mark(kind, s, &tok);
}

}  // namespace rt
}  // namespace cs
