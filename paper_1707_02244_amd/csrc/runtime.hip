// Host runtime and C ABI of the partial-circulant LASSO library.
//
// A plan per (device, n, d) holds the twiddle tables (computed in double
// precision with std::cos / std::sin and rounded to float) and the
// workspace: the four-step spectrum buffer Y (N = n/2 complex), the table of
// c_hat (N + 1 complex, bin k1 + N1*k2 at [k1*N2 + k2], Nyquist at [N]) and
// the table of DFT_n(P^T y) (same layout; its bins k' < m are y's m-point
// spectrum).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "cscirc.h"
#include "rt_common.hpp"
#include "launch.hpp"
#include "solve_persistent.hpp"
#include "unrolled.hpp"
#include "cpadmm.hpp"

#include <algorithm>
#include <numeric>

namespace cs {
namespace rt {

thread_local std::string g_err;

cs_status fail(cs_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

std::mutex g_mu;

int ilog2(int64_t v) {
  int r = 0;
  while ((int64_t(1) << r) < v) ++r;
  return r;
}
bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }

float2 root(int64_t e, int64_t L) {
  const double a = -2.0 * M_PI * double(e % L) / double(L);
  return make_float2(float(std::cos(a)), float(std::sin(a)));
}

__global__ void k_fill(float* __restrict__ p, size_t count, float v) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < count; i += stride) p[i] = v;
}

cs_status fill(float* p, size_t count, float v, hipStream_t s) {
  if (count == 0) return CS_OK;
  size_t blocks = (count + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  k_fill<<<dim3(unsigned(blocks)), dim3(256), 0, s>>>(p, count, v);
  CS_HIP(hipGetLastError());
  return CS_OK;
}

// Objective trace: block t adds the row-pass residual partials res[t][*]
// and the column-pass l1 partials l1[t][*] in a fixed order and writes
//   obj[t] = 1/(2m) sum res + lambda sum l1    (Eq. 3 halved, Parseval)
__global__ void k_objective(const double* __restrict__ res, int nres, const double* __restrict__ l1, int nl1,
                            double inv_2m, double lambda, float* __restrict__ obj) {
  __shared__ double r0[256], r1[256];
  const int t = blockIdx.x;
  const double* p0 = res + (size_t)t * nres;
  const double* p1 = l1 + (size_t)t * nl1;
  double a0 = 0.0, a1 = 0.0;
  for (int i = threadIdx.x; i < nres; i += 256) a0 += p0[i];
  for (int i = threadIdx.x; i < nl1; i += 256) a1 += p1[i];
  r0[threadIdx.x] = a0;
  r1[threadIdx.x] = a1;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (threadIdx.x < k) { r0[threadIdx.x] += r0[threadIdx.x + k]; r1[threadIdx.x] += r1[threadIdx.x + k]; }
    __syncthreads();
  }
  if (threadIdx.x == 0) obj[t] = float(inv_2m * r0[0] + lambda * r1[0]);
}

cs_status objective_reduce(const double* res, int nres, const double* l1, int nl1, double inv_2m,
                           double lambda, float* obj, int iters, hipStream_t s) {
  if (iters <= 0) return CS_OK;
  k_objective<<<dim3(iters), dim3(256), 0, s>>>(res, nres, l1, nl1, inv_2m, lambda, obj);
  CS_HIP(hipGetLastError());
  return CS_OK;
}

__global__ void k_max_abs2(const float2* __restrict__ t, int count, float* __restrict__ out) {
  __shared__ float red[256];
  float m = 0.0f;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x)
    m = fmaxf(m, cabs2(t[i]));
  red[threadIdx.x] = m;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (threadIdx.x < k) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + k]);
    __syncthreads();
  }
  // non-negative floats order like their bit patterns
  if (threadIdx.x == 0) atomicMax(reinterpret_cast<unsigned int*>(out), __float_as_uint(red[0]));
}

cs_status max_abs2(const float2* t, int count, float* out, hipStream_t s) {
  int blocks = (count + 255) / 256;
  if (blocks > 1024) blocks = 1024;
  if (blocks < 1) blocks = 1;
  k_max_abs2<<<dim3(blocks), dim3(256), 0, s>>>(t, count, out);
  CS_HIP(hipGetLastError());
  return CS_OK;
}

// Optional per-launch timing (diagnostics): each solver kernel launch is
// bracketed by two hipEvents on its own stream.
struct TimedLaunch {
  int kind;
  hipEvent_t start, stop;
};
std::mutex g_tmu;
bool g_timing = false;
std::vector<TimedLaunch> g_timed;
std::vector<TimedLaunch> g_open;
std::vector<hipEvent_t> g_event_pool;
const char* kTimedNames[T_COUNT] = {"passA_ista", "passB_ista", "passA_admm", "passB_admm",
                                    "solve_ista", "solve_admm", "batched",
                                    "col2_ista", "row2_ista", "col2_admm", "row2_admm", "direct",
                                    "direct_T", "cp_row", "cp_col"};

hipEvent_t take_event() {
  if (!g_event_pool.empty()) {
    hipEvent_t e = g_event_pool.back();
    g_event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

bool timing_on() {
  std::lock_guard<std::mutex> lk(g_tmu);
  return g_timing;
}

hipError_t timed_mark(int kind, hipStream_t s, long* tok) {
  std::lock_guard<std::mutex> lk(g_tmu);
  if (*tok < 0) {
    TimedLaunch t{kind, take_event(), take_event()};
    if (!t.start || !t.stop) return hipErrorOutOfMemory;
    hipError_t e = hipEventRecord(t.start, s);
    if (e != hipSuccess) return e;
    *tok = long(g_open.size());
    g_open.push_back(t);
    return hipSuccess;
  }
  TimedLaunch t = g_open[size_t(*tok)];
  g_open.erase(g_open.begin() + *tok);
  hipError_t e = hipEventRecord(t.stop, s);
  if (e != hipSuccess) return e;
  g_timed.push_back(t);
  return hipSuccess;
}

}  // namespace rt

namespace {
using namespace rt;

constexpr int64_t kMinN = 64;
constexpr int64_t kCpMinN = 256;   // circulant ADMM with an arbitrary row set
constexpr int64_t kMaxN = int64_t(1) << 26;
constexpr int64_t kMaxNUnrolled = int64_t(1) << 25;
constexpr int64_t kCpMaxN = int64_t(1) << 22;   // circulant ADMM with an arbitrary row set
constexpr int kMinLogNPersistent = 7;    // N = n/2 = 2^7 .. 2^21: one cooperative launch per solve
constexpr int kMaxLogNPersistent = 21;

// 0: choose per size; 1: two launches per iteration; 2: persistent launch
int g_path = 0;

// Bound of one grid-barrier wait of the persistent solver.  A real wait
// lasts a few microseconds; a wait that reaches the bound sets the plan's
// error flag (reported by cs_check_device) and the launch drains.
constexpr uint64_t kBarWaitMs = 20;

// A plan for (n, d): the four-step geometry and one block of device memory
// holding, in this order (float2 units, each part rounded up to 64):
//   barrier area   grid-barrier counters and the error flag (kBarWords words;
//                  first, so the flag sits at the block's start for every n)
//   scal           small device scalars
//   twiddles       W_N1, W_N2, W_N^e (two levels), W_n^k1, W_2N2^p
//   Y              the four-step spectrum buffer (N complex)
//   chat, yhat     the c_hat and DFT_n(P^T y) tables (N + 1 complex each)
// The block is the library's own allocation (cached per device, n, d), a
// caller's workspace (cs_set_workspace) or the allocation-free entry point's
// scratch array; `bind` points a plan at it.
struct Plan {
  int dev = 0;
  int64_t n = 0;
  int d = 0;
  int N = 0, N1 = 0, N2 = 0, M = 0, lo_bits = 0, logN = 0;
  bool persistent[2][5][2] = {};   // [alg][d/2 index][traced]: cooperative launch fits
  uint64_t bar_ticks = 0;       // bound of one grid-barrier wait (device wall-clock ticks)
  int64_t oB = 0, oS = 0, oT1 = 0, oT2 = 0, oLo = 0, oHi = 0, oK1 = 0, oP = 0, oY = 0, oC = 0, oYh = 0;
  size_t bytes = 0;             // size of the memory block
  float2* mem = nullptr;        // the block (nullptr: not bound)
  unsigned* bar = nullptr;      // grid barrier counters, error flag at [kBarErr]
  float2 *Y = nullptr, *chat = nullptr, *yhat = nullptr;
  float2 *tw1 = nullptr, *tw2 = nullptr, *twlo = nullptr, *twhi = nullptr;
  float2 *twk1 = nullptr, *twp = nullptr;
  float* scal = nullptr;    // small device scalars (norm bound)
};

// Plans and workspaces live until the process ends and are never destroyed:
// the caches are heap objects that are never deleted, so no destructor calls
// into the HIP runtime during static destruction (by then the runtime, or a
// profiler wrapped around it, may already be finalised).  The device memory is
// returned with the process.
auto& g_plans = *new std::map<std::tuple<int, int64_t, int>, std::unique_ptr<Plan>>();

int solve_blocks_per_cu_dispatch(int logN, int alg, int d2, bool tr) {
  switch (logN) {
#define CS_CASE(L) case L: return tr ? solve_blocks_per_cu<L, true>(alg, d2) : solve_blocks_per_cu<L, false>(alg, d2);
    CS_CASE(7) CS_CASE(8) CS_CASE(9) CS_CASE(10) CS_CASE(11) CS_CASE(12) CS_CASE(13) CS_CASE(14)
    CS_CASE(15) CS_CASE(16) CS_CASE(17) CS_CASE(18) CS_CASE(19) CS_CASE(20) CS_CASE(21)
#undef CS_CASE
    default: return 0;
  }
}

hipError_t launch_solve_dispatch(int logN, int alg, int d2, bool tr, const SolveArgs& a, hipStream_t s) {
  switch (logN) {
#define CS_CASE(L) case L: return tr ? launch_solve<L, true>(alg, d2, a, s) : launch_solve<L, false>(alg, d2, a, s);
    CS_CASE(7) CS_CASE(8) CS_CASE(9) CS_CASE(10) CS_CASE(11) CS_CASE(12) CS_CASE(13) CS_CASE(14)
    CS_CASE(15) CS_CASE(16) CS_CASE(17) CS_CASE(18) CS_CASE(19) CS_CASE(20) CS_CASE(21)
#undef CS_CASE
    default: return hipErrorInvalidValue;
  }
}

// Per-device facts the plans need, queried once into fixed arrays (no heap
// allocation, so the allocation-free entry point can use them): the CU
// count, the wall-clock rate and whether each persistent-solver instance fits
// as one cooperative launch.
constexpr int kMaxDevices = 64;
struct DevInfo {
  bool ready = false;
  int cus = 0;
  uint64_t bar_ticks = 0;
  bool persistent[kMaxLogNPersistent + 1][2][4][2] = {};   // [log2 N][alg][log2 (d/2)][traced]
};
DevInfo g_dev[kMaxDevices];

cs_status dev_info(int dev, const DevInfo** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(CS_ENOTSUP, "device %d beyond the supported %d", dev, kMaxDevices);
  DevInfo& di = g_dev[dev];
  if (!di.ready) {
    int khz = 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0) khz = 100000;
    // one barrier wait may last at most kBarWaitMs of device wall-clock time
    di.bar_ticks = uint64_t(khz) * kBarWaitMs;
    CS_HIP(hipDeviceGetAttribute(&di.cus, hipDeviceAttributeMultiprocessorCount, dev));
    for (int L = kMinLogNPersistent; L <= kMaxLogNPersistent; ++L) {
      const int N1 = (L % 2) ? (1 << ((L - 1) / 2)) : (1 << (L / 2 - 1));
      const int N2 = (1 << L) / N1;
      for (int alg = 0; alg < 2; ++alg)
        for (int k = 0; k < 4; ++k)
          for (int tr = 0; tr < 2; ++tr) {
            const int nb = solve_blocks_per_cu_dispatch(L, alg, 1 << k, tr != 0);
            di.persistent[L][alg][k][tr] = nb >= 1 && int64_t(nb) * di.cus >= N2 / kColsPerBlock;
          }
    }
    di.ready = true;
  }
  *out = &di;
  return CS_OK;
}

// Geometry and memory layout of the (n, d) plan (no device query).
void plan_layout(int64_t n, int d, Plan& p) {
  p.n = n;
  p.d = d;
  p.N = int(n / 2);
  const int pN = ilog2(p.N);
  p.logN = pN;
  // four-step split: odd log2 N -> N2 = 2 N1, even -> N2 = 4 N1 (so the
  // persistent solver's grid N2/8 owns N1/2 row pairs in 2 or 1 per group)
  p.N1 = (pN % 2) ? (1 << ((pN - 1) / 2)) : (1 << (pN / 2 - 1));
  p.N2 = p.N / p.N1;
  p.M = int((n / d) / p.N1);
  p.lo_bits = (pN + 1) / 2;
  const int64_t nlo = int64_t(1) << p.lo_bits, nhi = int64_t(p.N) >> p.lo_bits;
  auto up = [](int64_t v) { return (v + 63) & ~int64_t(63); };
  p.oB = 0;
  p.oS = p.oB + up(kBarWords / 2);
  p.oT1 = p.oS + 64;
  p.oT2 = p.oT1 + up(p.N1);
  p.oLo = p.oT2 + up(p.N2);
  p.oHi = p.oLo + up(nlo);
  p.oK1 = p.oHi + up(nhi);
  p.oP = p.oK1 + up(p.N1);
  p.oY = p.oP + up(p.N2);
  p.oC = p.oY + up(p.N);
  p.oYh = p.oC + up(p.N + 1);
  p.bytes = size_t(p.oYh + up(p.N + 1)) * sizeof(float2);
}

// Geometry, layout and device facts of the (n, d) plan; binds no memory.
// Call with g_mu held.
cs_status plan_geometry(int dev, int64_t n, int d, Plan& p) {
  const DevInfo* di = nullptr;
  cs_status st = dev_info(dev, &di);
  if (st != CS_OK) return st;
  plan_layout(n, d, p);
  p.dev = dev;
  p.bar_ticks = di->bar_ticks;
  for (int alg = 0; alg < 2; ++alg)
    for (int k = 0; k < 4; ++k)
      for (int tr = 0; tr < 2; ++tr)
        p.persistent[alg][k][tr] = p.logN >= kMinLogNPersistent && p.logN <= kMaxLogNPersistent &&
                                   di->persistent[p.logN][alg][k][tr];
  return CS_OK;
}

void bind(Plan& p, float2* b) {
  p.mem = b;
  p.bar = reinterpret_cast<unsigned*>(b + p.oB);
  p.scal = reinterpret_cast<float*>(b + p.oS);
  p.tw1 = b + p.oT1; p.tw2 = b + p.oT2; p.twlo = b + p.oLo; p.twhi = b + p.oHi;
  p.twk1 = b + p.oK1; p.twp = b + p.oP;
  p.Y = b + p.oY; p.chat = b + p.oC; p.yhat = b + p.oYh;
}

// Twiddle tables of a plan computed on the device (double precision, rounded
// to float), for memory the library does not fill from the host.
__global__ void k_twiddles(float2* __restrict__ tw1, float2* __restrict__ tw2, float2* __restrict__ twlo,
                           float2* __restrict__ twhi, float2* __restrict__ twk1, float2* __restrict__ twp,
                           int N1, int N2, int lo_bits, int64_t N, int64_t n) {
  const int64_t nlo = int64_t(1) << lo_bits, nhi = N >> lo_bits;
  auto rt = [](int64_t e, int64_t L) {
    double s_, c_;
    sincos(-2.0 * M_PI * double(e % L) / double(L), &s_, &c_);
    return make_float2(float(c_), float(s_));
  };
  const int64_t total = int64_t(N1) + N2 + nlo + nhi + N1 + N2;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < total; i += int64_t(gridDim.x) * blockDim.x) {
    int64_t k = i;
    if (k < N1) { tw1[k] = rt(k, N1); continue; }
    k -= N1;
    if (k < N2) { tw2[k] = rt(k, N2); continue; }
    k -= N2;
    if (k < nlo) { twlo[k] = rt(k, N); continue; }
    k -= nlo;
    if (k < nhi) { twhi[k] = rt(k * nlo, N); continue; }
    k -= nhi;
    if (k < N1) { twk1[k] = rt(k, n); continue; }
    k -= N1;
    twp[k] = rt(k, 2 * int64_t(N2));
  }
}

cs_status device_twiddles(const Plan& p, hipStream_t s) {
  const int64_t total = int64_t(p.N1) * 2 + int64_t(p.N2) * 2 + (int64_t(1) << p.lo_bits) + (int64_t(p.N) >> p.lo_bits);
  const unsigned blocks = unsigned(std::min<int64_t>((total + 255) / 256, 1024));
  k_twiddles<<<dim3(blocks), dim3(256), 0, s>>>(p.tw1, p.tw2, p.twlo, p.twhi, p.twk1, p.twp, p.N1, p.N2,
                                                p.lo_bits, int64_t(p.N), p.n);
  CS_HIP(hipGetLastError());
  return CS_OK;
}

// The library's own plan for (current device, n, d), allocated and filled
// on first use and cached.
cs_status get_plan(int64_t n, int d, Plan** out) {
  int dev = 0;
  CS_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_mu);
  auto key = std::make_tuple(dev, n, d);
  auto it = g_plans.find(key);
  if (it != g_plans.end()) {
    *out = it->second.get();
    return CS_OK;
  }
  auto p = std::make_unique<Plan>();
  cs_status st = plan_geometry(dev, n, d, *p);
  if (st != CS_OK) return st;
  float2* b = nullptr;
  hipError_t e = hipMalloc(&b, p->bytes);
  if (e != hipSuccess) return fail(CS_ENOMEM, "hipMalloc of %zu bytes for plan n=%lld d=%d failed: %s",
                                   p->bytes, (long long)n, d, hipGetErrorString(e));
  bind(*p, b);
  // barrier area, scalars and twiddle tables from the host (zeros for the
  // first two)
  const int64_t nlo = int64_t(1) << p->lo_bits, nhi = int64_t(p->N) >> p->lo_bits;
  std::vector<float2> h(size_t(p->oY), make_float2(0.f, 0.f));
  auto put = [&](int64_t off, int64_t cnt, auto fn) {
    for (int64_t i = 0; i < cnt; ++i) h[size_t(off + i)] = fn(i);
  };
  put(p->oT1, p->N1, [&](int64_t i) { return root(i, p->N1); });
  put(p->oT2, p->N2, [&](int64_t i) { return root(i, p->N2); });
  put(p->oLo, nlo, [&](int64_t i) { return root(i, p->N); });
  put(p->oHi, nhi, [&](int64_t i) { return root(i * nlo, p->N); });
  put(p->oK1, p->N1, [&](int64_t i) { return root(i, n); });
  put(p->oP, p->N2, [&](int64_t i) { return root(i, 2 * int64_t(p->N2)); });
  e = hipMemcpy(b, h.data(), h.size() * sizeof(float2), hipMemcpyHostToDevice);
  if (e != hipSuccess) return fail(CS_EHIP, "hipMemcpy of plan tables failed: %s", hipGetErrorString(e));
  *out = p.get();
  g_plans[key] = std::move(p);
  return CS_OK;
}

// Memory blocks the caller provides: a workspace set by cs_set_workspace per
// device, and the allocation-free entry point's scratch array.  `tables_n` is
// the n whose twiddle tables the block holds (0: none yet); a block whose
// barrier area has not been cleared yet has `cleared` false.
struct ExtBlock {
  void* ptr = nullptr;
  size_t bytes = 0;
  int64_t tables_n = 0;
  bool cleared = false;
};
ExtBlock g_ws[kMaxDevices];

// A plan for (n, d) bound to an external block: geometry from plan_geometry,
// twiddle tables computed on the stream when the block holds another n's,
// barrier area (counters and error flag) cleared on the block's first use.
// Call with g_mu held.
cs_status bind_external(int dev, int64_t n, int d, ExtBlock& blk, hipStream_t s, Plan& p) {
  cs_status st = plan_geometry(dev, n, d, p);
  if (st != CS_OK) return st;
  if (p.bytes > blk.bytes)
    return fail(CS_EINVAL, "workspace of %zu bytes is too small for n=%lld d=%d (needs %zu bytes)", blk.bytes,
                (long long)n, d, p.bytes);
  bind(p, static_cast<float2*>(blk.ptr));
  if (!blk.cleared) {
    if ((st = fill(reinterpret_cast<float*>(p.bar), kBarWords, 0.0f, s)) != CS_OK) return st;
    blk.cleared = true;
  }
  if (blk.tables_n != n) {
    if ((st = device_twiddles(p, s)) != CS_OK) return st;
    blk.tables_n = n;
  }
  return CS_OK;
}

// Allocation-free ISTA (cs_ista_solve_noalloc): its plan block is the
// file-scope device array `scratch`, sized for the largest supported n.  The
// array's name is a host-side stand-in in host code; its device address is
// taken once per device with hipGetSymbolAddress (with that device current)
// and kept in g_noalloc[dev].ptr, which is what every kernel receives.
constexpr int64_t kNoAllocMaxN = int64_t(1) << 20;
constexpr int64_t up64c(int64_t v) { return (v + 63) & ~int64_t(63); }
constexpr int ilog2cc(int64_t v) { return v <= 1 ? 0 : 1 + ilog2cc(v / 2); }
// float2 words of the (n, d) plan block: the layout of plan_layout
constexpr int64_t layout_words(int64_t n) {
  const int64_t N = n / 2;
  const int pN = ilog2cc(N);
  const int64_t N1 = (pN % 2) ? (int64_t(1) << ((pN - 1) / 2)) : (int64_t(1) << (pN / 2 - 1));
  const int64_t N2 = N / N1;
  const int lo = (pN + 1) / 2;
  return up64c(kBarWords / 2) + 64 + up64c(N1) + up64c(N2) + up64c(int64_t(1) << lo) + up64c(N >> lo) +
         up64c(N1) + up64c(N2) + up64c(N) + 2 * up64c(N + 1);
}
constexpr int64_t kNoAllocWords = layout_words(kNoAllocMaxN);
static __device__ __align__(256) float2 scratch[kNoAllocWords];
ExtBlock g_noalloc[kMaxDevices];

// The plan a single-signal call runs on: bound to the device's workspace if
// the caller has set one, else the library's cached plan.  `cached` (may be
// null) receives the library plan when one is used (it owns the objective
// buffer).
// The external blocks of a device whose error flags cs_check_device reads.
std::vector<ExtBlock*> ext_blocks(int dev) { return {&g_ws[dev], &g_noalloc[dev]}; }

cs_status plan_for_call(int64_t n, int d, hipStream_t s, Plan& view, Plan** cached) {
  int dev = 0;
  CS_HIP(hipGetDevice(&dev));
  if (dev >= 0 && dev < kMaxDevices) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_ws[dev].ptr) {
      if (cached) *cached = nullptr;
      return bind_external(dev, n, d, g_ws[dev], s, view);
    }
  }
  Plan* P = nullptr;
  cs_status st = get_plan(n, d, &P);
  if (st != CS_OK) return st;
  view = *P;
  if (cached) *cached = P;
  return CS_OK;
}

// ---------------------------------------------------------------------------
hipError_t launchA(const Plan& P, int op, const PassAArgs& a, hipStream_t s) {
  const int grid = P.N1 / 2;
  const int d2 = P.d / 2;
  switch (P.N2) {
    case 8: return launch_passA<8>(op, d2, grid, a, s);
    case 16: return launch_passA<16>(op, d2, grid, a, s);
    case 32: return launch_passA<32>(op, d2, grid, a, s);
    case 64: return launch_passA<64>(op, d2, grid, a, s);
    case 128: return launch_passA<128>(op, d2, grid, a, s);
    case 256: return launch_passA<256>(op, d2, grid, a, s);
    case 512: return launch_passA<512>(op, d2, grid, a, s);
    case 1024: return launch_passA<1024>(op, d2, grid, a, s);
    case 2048: return launch_passA<2048>(op, d2, grid, a, s);
    case 4096: return launch_passA<4096>(op, d2, grid, a, s);
    case 8192: return launch_passA<8192>(op, d2, grid, a, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launchCpRow(const Plan& P, const CpArgs& a, hipStream_t s) {
  const int grid = P.N1 / 2;
  switch (P.N2) {
    case 16: return launch_cp_row<16>(grid, a, s);
    case 32: return launch_cp_row<32>(grid, a, s);
    case 64: return launch_cp_row<64>(grid, a, s);
    case 128: return launch_cp_row<128>(grid, a, s);
    case 256: return launch_cp_row<256>(grid, a, s);
    case 512: return launch_cp_row<512>(grid, a, s);
    case 1024: return launch_cp_row<1024>(grid, a, s);
    case 2048: return launch_cp_row<2048>(grid, a, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launchCpCol(const Plan& P, int last, const CpArgs& a, hipStream_t s) {
  const int grid = P.N2 / cp_cb(P.N1);
  switch (P.N1) {
    case 8: return launch_cp_col<8>(last, grid, a, s);
    case 16: return launch_cp_col<16>(last, grid, a, s);
    case 32: return launch_cp_col<32>(last, grid, a, s);
    case 64: return launch_cp_col<64>(last, grid, a, s);
    case 128: return launch_cp_col<128>(last, grid, a, s);
    case 256: return launch_cp_col<256>(last, grid, a, s);
    case 512: return launch_cp_col<512>(last, grid, a, s);
    case 1024: return launch_cp_col<1024>(last, grid, a, s);
    default: return hipErrorInvalidValue;
  }
}

// P^T y (zero elsewhere) and the indicator of Omega, for the circulant ADMM
// with an arbitrary row set, into their column-blocked arrays: sample j is
// component j mod 2 of pair p = j / 2 = i N2 + j2, stored at pair
// ((j2 / CB) N1 + i) CB + j2 mod CB.  omega is read from `idx` (int32,
// validated on the host); both arrays are zeroed first by the caller.
__global__ void k_cp_scatter(const int* __restrict__ idx, int64_t m, const float* __restrict__ y, int N1, int N2,
                             int CB, float* __restrict__ py, float* __restrict__ om) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < m; i += int64_t(gridDim.x) * blockDim.x) {
    const int j = idx[i];
    const int p = j >> 1, r = p / N2, j2 = p % N2;
    const int64_t pb = (int64_t(j2 / CB) * N1 + r) * CB + j2 % CB;
    py[2 * pb + (j & 1)] = y[i];
    om[2 * pb + (j & 1)] = 1.0f;
  }
}

// Generator of C B for the order-L box blur B (Section 7): the mean of c
// over the L samples starting at k, circularly (n a power of two), summed in
// double and rounded once.  Neighbouring threads read overlapping windows,
// so the L-fold reads hit the cache.
__global__ void k_box_blur(const float* __restrict__ c, int64_t n, int L, float* __restrict__ out) {
  const int64_t mask = n - 1;
  const double inv = 1.0 / double(L);
  for (int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; k < n; k += int64_t(gridDim.x) * blockDim.x) {
    double s = 0.0;
    for (int t = 0; t < L; ++t) s += double(c[(k + t) & mask]);
    out[k] = float(s * inv);
  }
}

hipError_t launchB(const Plan& P, int mode, const PassBArgs& a, hipStream_t s) {
  const int grid = P.N2 / pass_b_cols(P.N1);
  switch (P.N1) {
    case 4: return launch_passB<4>(mode, grid, a, s);
    case 8: return launch_passB<8>(mode, grid, a, s);
    case 16: return launch_passB<16>(mode, grid, a, s);
    case 32: return launch_passB<32>(mode, grid, a, s);
    case 64: return launch_passB<64>(mode, grid, a, s);
    case 128: return launch_passB<128>(mode, grid, a, s);
    case 256: return launch_passB<256>(mode, grid, a, s);
    case 512: return launch_passB<512>(mode, grid, a, s);
    case 1024: return launch_passB<1024>(mode, grid, a, s);
    case 2048: return launch_passB<2048>(mode, grid, a, s);
    case 4096: return launch_passB<4096>(mode, grid, a, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launchUA(const Plan& P, int op, int batch, const PassAArgs& a, const UStride& st, hipStream_t s) {
  const int grid = P.N1 / 2 / urow_pairs(P.N2);
  const int d2 = P.d / 2;
  switch (P.N2) {
#define CS_CASE(L) case L: return launch_urow<L>(op, d2, grid, batch, a, st, s);
    CS_CASE(8) CS_CASE(16) CS_CASE(32) CS_CASE(64) CS_CASE(128) CS_CASE(256) CS_CASE(512) CS_CASE(1024)
    CS_CASE(2048) CS_CASE(4096) CS_CASE(8192)
#undef CS_CASE
    default: return hipErrorInvalidValue;
  }
}

hipError_t launchUB(const Plan& P, int mode, int batch, const PassBArgs& a, const UStride& st, hipStream_t s) {
  const int grid = P.N2 / ucol_cols(P.N1);
  switch (P.N1) {
#define CS_CASE(L) case L: return launch_ucol<L>(mode, grid, batch, a, st, s);
    CS_CASE(4) CS_CASE(8) CS_CASE(16) CS_CASE(32) CS_CASE(64) CS_CASE(128) CS_CASE(256) CS_CASE(512) CS_CASE(1024)
    CS_CASE(2048)
#undef CS_CASE
    default: return hipErrorInvalidValue;
  }
}

PassAArgs argsA(const Plan& P) {
  PassAArgs a{};
  a.Y = P.Y; a.chat = P.chat; a.yhat = P.yhat; a.table = nullptr;
  a.tw2 = P.tw2; a.twk1 = P.twk1; a.twp = P.twp;
  a.N1 = P.N1; a.M = P.M; a.N = P.N;
  a.inv_n = float(1.0 / double(P.n));
  a.inv_d = float(1.0 / double(P.d));
  return a;
}

PassBArgs argsB(const Plan& P) {
  PassBArgs b{};
  b.Y = P.Y; b.tw1 = P.tw1; b.twlo = P.twlo; b.twhi = P.twhi; b.lo_bits = P.lo_bits;
  b.N2 = P.N2; b.N = P.N; b.d = P.d;
  return b;
}


// c_hat table from c (pass B forward on the real signal, pass A split).
cs_status setup_chat(const Plan& P, const float* c, hipStream_t s) {
  PassBArgs b = argsB(P);
  b.in0 = c;
  CS_LAUNCH(launchB(P, B_FWD_REAL, b, s));
  PassAArgs a = argsA(P);
  a.table = P.chat;
  CS_LAUNCH(launchA(P, A_SPEC, a, s));
  return CS_OK;
}

// DFT_n(P^T y) table (its first m bins are the m-point spectrum of y).
cs_status setup_yhat(const Plan& P, const float* y, hipStream_t s) {
  PassBArgs b = argsB(P);
  b.in0 = y;
  CS_LAUNCH(launchB(P, B_FWD_UP, b, s));
  PassAArgs a = argsA(P);
  a.table = P.yhat;
  CS_LAUNCH(launchA(P, A_SPEC, a, s));
  return CS_OK;
}

// Whether this solve runs as one cooperative launch.
cs_status use_persistent(const Plan& P, int alg, bool traced, bool* out) {
  // d = 1 (single-bin classes) runs the two-launch schedule only
  const bool fits = P.d >= 2 && P.persistent[alg][ilog2(P.d / 2)][traced ? 1 : 0];
  if (g_path == 2 && !fits)
    return fail(CS_ENOTSUP, "persistent solver not available for n=%lld d=%d", (long long)P.n, P.d);
  *out = (g_path == 2) || (g_path == 0 && fits);
  return CS_OK;
}

SolveArgs solve_args(const Plan& P) {
  SolveArgs a{};
  a.Y = P.Y; a.chat = P.chat; a.yhat = P.yhat;
  a.tw1 = P.tw1; a.tw2 = P.tw2; a.twlo = P.twlo; a.twhi = P.twhi; a.twk1 = P.twk1; a.twp = P.twp;
  a.lo_bits = P.lo_bits;
  a.bar = P.bar; a.err = reinterpret_cast<int*>(P.bar + kBarErr);
  a.max_ticks = P.bar_ticks;
  a.inv_n = float(1.0 / double(P.n));
  a.inv_d = float(1.0 / double(P.d));
  return a;
}

cs_status check_common(const void* c, int64_t n, int d) {
  if (!c) return fail(CS_EINVAL, "c is NULL");
  if (!is_pow2(n) || n < kMinN || n > kMaxN)
    return fail(CS_EINVAL, "n=%lld must be a power of two in [%lld, %lld]", (long long)n,
                (long long)kMinN, (long long)kMaxN);
  if (d != 1 && d != 2 && d != 4 && d != 8 && d != 16)
    return fail(CS_EINVAL, "d=%d must be 1, 2, 4, 8 or 16", d);
  return CS_OK;
}

bool finite(float v) { return std::isfinite(v); }

// Gradients from the partial sums: block t adds the `count` partials of
// step t (layout part[t][q][count]) in a fixed order and applies
//   lambar_t = tau_t S0,  taubar_t = lam_t S0 + S1 / tau_t.
__global__ void k_unrolled_grads(const double* __restrict__ part, int count, const float* __restrict__ tau,
                                 const float* __restrict__ lam, float* __restrict__ g_lam,
                                 float* __restrict__ g_tau) {
  __shared__ double r0[256], r1[256];
  const int t = blockIdx.x;
  const double* p0 = part + (size_t)t * 2 * count;
  const double* p1 = p0 + count;
  double a0 = 0.0, a1 = 0.0;
  for (int i = threadIdx.x; i < count; i += 256) { a0 += p0[i]; a1 += p1[i]; }
  r0[threadIdx.x] = a0;
  r1[threadIdx.x] = a1;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (threadIdx.x < k) { r0[threadIdx.x] += r0[threadIdx.x + k]; r1[threadIdx.x] += r1[threadIdx.x + k]; }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double tt = tau[t], ll = lam[t];
    g_lam[t] = float(tt * r0[0]);
    g_tau[t] = float(ll * r0[0] + r1[0] / tt);
  }
}

// Partial-sum buffers of an objective trace over `iters` iterations:
// res[iters][N1/2] (one per row-pass workgroup), then l1[iters][N2/8].  One
// grow-only buffer per device, shared by traced solves on that device.
struct ObjBuf {
  double* p = nullptr;
  size_t cap = 0;
};
ObjBuf g_obj[kMaxDevices];

cs_status get_objbuf(const Plan& P, int iters, double** res, double** l1, hipStream_t s) {
  const size_t nres = size_t(P.N1 / 2), nl1 = size_t(P.N2 / pass_b_cols(P.N1));
  const size_t need = size_t(iters) * (nres + nl1);
  if (P.dev < 0 || P.dev >= kMaxDevices) return fail(CS_ENOTSUP, "device %d beyond the supported range", P.dev);
  std::lock_guard<std::mutex> lk(g_mu);
  ObjBuf& B = g_obj[P.dev];
  if (B.cap < need) {
    CS_HIP(hipStreamSynchronize(s));
    if (B.p) CS_HIP(hipFree(B.p));
    B.p = nullptr;
    B.cap = 0;
    hipError_t e = hipMalloc(&B.p, need * sizeof(double));
    if (e != hipSuccess) return fail(CS_ENOMEM, "hipMalloc of %zu bytes for the objective trace failed",
                                     need * sizeof(double));
    B.cap = need;
  }
  *res = B.p;
  *l1 = B.p + size_t(iters) * nres;
  return CS_OK;
}

// Working memory of the circulant ADMM with an arbitrary row set: the
// interleaved spectrum buffer of both signals (n complex) and the
// column-blocked mu, nu, P^T y and Omega indicator (n/2 pairs each).  One
// grow-only buffer per device.
struct CpBuf {
  float2* p = nullptr;
  size_t cap = 0;   // float2 elements
};
CpBuf g_cp[kMaxDevices];

cs_status get_cpbuf(const Plan& P, float2** out, hipStream_t s) {
  const size_t need = size_t(P.n) + 4 * size_t(P.N);
  if (P.dev < 0 || P.dev >= kMaxDevices) return fail(CS_ENOTSUP, "device %d beyond the supported range", P.dev);
  std::lock_guard<std::mutex> lk(g_mu);
  CpBuf& B = g_cp[P.dev];
  if (B.cap < need) {
    CS_HIP(hipStreamSynchronize(s));
    if (B.p) CS_HIP(hipFree(B.p));
    B.p = nullptr;
    B.cap = 0;
    hipError_t e = hipMalloc(&B.p, need * sizeof(float2));
    if (e != hipSuccess) return fail(CS_ENOMEM, "hipMalloc of %zu bytes for the circulant ADMM failed",
                                     need * sizeof(float2));
    B.cap = need;
  }
  *out = B.p;
  return CS_OK;
}

// Unrolled ISTA workspace per (device, n, d, batch, checkpoint interval):
// spectrum buffers, y_hat and ybar tables and time-domain state of every
// signal, the records of one segment, and the partial sums (grown with K).
struct UPlan {
  float2 *Y = nullptr, *yhat = nullptr, *ybar = nullptr;
  float *xs = nullptr, *rv = nullptr, *rd = nullptr, *xbar = nullptr, *vbar = nullptr;
  double* part = nullptr;
  size_t part_cap = 0;
  void* mem = nullptr;
};
auto& g_uplans = *new std::map<std::tuple<int, int64_t, int, int, int>, std::unique_ptr<UPlan>>();

int64_t ckpt_count(int K, int every) { return K > 0 ? (K - 1) / every : 0; }

cs_status get_uplan(const Plan& P, int Bt, int every, int K, UPlan** out) {
  std::lock_guard<std::mutex> lk(g_mu);
  auto key = std::make_tuple(P.dev, P.n, P.d, Bt, every);
  auto& slot = g_uplans[key];
  if (!slot) {
    auto u = std::make_unique<UPlan>();
    const size_t N = size_t(P.N), n = size_t(P.n), B = size_t(Bt), E = size_t(every);
    const size_t bytes = (B * N + 2 * B * (N + 1)) * sizeof(float2) + (3 * B * n + 2 * E * B * n) * sizeof(float) + 1024;
    hipError_t e = hipMalloc(&u->mem, bytes);
    if (e != hipSuccess) return fail(CS_ENOMEM, "hipMalloc of %zu bytes for the unrolled workspace failed", bytes);
    char* p = static_cast<char*>(u->mem);
    auto take = [&](size_t b) { char* r = p; p += (b + 255) & ~size_t(255); return r; };
    u->Y = reinterpret_cast<float2*>(take(B * N * sizeof(float2)));
    u->yhat = reinterpret_cast<float2*>(take(B * (N + 1) * sizeof(float2)));
    u->ybar = reinterpret_cast<float2*>(take(B * (N + 1) * sizeof(float2)));
    u->xs = reinterpret_cast<float*>(take(B * n * sizeof(float)));
    u->xbar = reinterpret_cast<float*>(take(B * n * sizeof(float)));
    u->vbar = reinterpret_cast<float*>(take(B * n * sizeof(float)));
    u->rv = reinterpret_cast<float*>(take(E * B * n * sizeof(float)));
    u->rd = reinterpret_cast<float*>(take(E * B * n * sizeof(float)));
    slot = std::move(u);
  }
  UPlan* u = slot.get();
  const size_t need = size_t(K) * 2 * size_t(Bt) * size_t(P.N2 / ucol_cols(P.N1));
  if (u->part_cap < need) {
    if (u->part) (void)hipFree(u->part);
    u->part = nullptr;
    u->part_cap = 0;
    hipError_t e = hipMalloc(&u->part, need * sizeof(double));
    if (e != hipSuccess) return fail(CS_ENOMEM, "hipMalloc of unrolled partial sums failed");
    u->part_cap = need;
  }
  *out = u;
  return CS_OK;
}

cs_status check_unrolled(const float* c, int64_t n, int d, int Bt, const float* y, const float* lam,
                         const float* tau, int K, int every) {
  cs_status st = check_common(c, n, d);
  if (st != CS_OK) return st;
  if (d < 2) return fail(CS_EINVAL, "d=%d: the unrolled solver needs d >= 2", d);
  if (n > kMaxNUnrolled) return fail(CS_EINVAL, "n=%lld: the unrolled solver takes n <= 2^25", (long long)n);
  if (!y || !lam || !tau) return fail(CS_EINVAL, "y, lam or tau is NULL");
  if (Bt < 1 || Bt > 65535) return fail(CS_EINVAL, "batch=%d must be in [1, 65535]", Bt);
  if (K < 1) return fail(CS_EINVAL, "K=%d must be >= 1", K);
  if (every < 1) return fail(CS_EINVAL, "every=%d must be >= 1", every);
  return CS_OK;
}

cs_status check_ista(const float* c, int64_t n, int d, const float* y, float lambda, float tau, int iters,
                     const float* x) {
  cs_status st = check_common(c, n, d);
  if (st != CS_OK) return st;
  if (!y || !x) return fail(CS_EINVAL, "y or x is NULL");
  if (!finite(lambda) || lambda < 0.0f) return fail(CS_EINVAL, "lambda=%g must be finite and >= 0", lambda);
  if (!finite(tau) || tau <= 0.0f) return fail(CS_EINVAL, "tau=%g must be finite and > 0", tau);
  if (iters < 0) return fail(CS_EINVAL, "iters=%d must be >= 0", iters);
  return CS_OK;
}

// Launch with per-launch timing when `timing` (diagnostics) is allowed.
template <class F>
hipError_t maybe_timed(bool timing, int kind, hipStream_t s, F&& launch) {
  return timing ? timed(kind, s, launch) : launch();
}

// ISTA (Alg. 1) on the plan V for iters >= 1: the c_hat / y_hat tables, then
// one persistent launch or two launches per iteration (always two with an
// objective trace).  `timing`: the launches may be bracketed by the timing
// events (which the library creates on first use).
cs_status ista_run(const Plan& V, const float* c, const float* y, float lambda, float tau, int iters, float* x,
                   float* obj, hipStream_t s, bool timing) {
  const Plan* P = &V;
  const int64_t n = V.n;
  const int d = V.d;
  cs_status st = CS_OK;
  if ((st = setup_chat(*P, c, s)) != CS_OK) return st;
  if ((st = setup_yhat(*P, y, s)) != CS_OK) return st;
  bool pers = false;
  if ((st = use_persistent(*P, 0, obj != nullptr, &pers)) != CS_OK) return st;
  if (pers) {
    // barrier counters start at zero (bit pattern of 0.0f); the error flag is
    // cleared by cs_check_device
    if ((st = fill(reinterpret_cast<float*>(P->bar), kBarErr, 0.0f, s)) != CS_OK) return st;
    SolveArgs sa = solve_args(*P);
    sa.x = x;
    sa.iters = iters;
    sa.tau = tau;
    sa.thr = tau * lambda;
    // objective trace: one residual and one l1 partial per workgroup and
    // iteration (G = N2 / 8 workgroups), reduced after the launch
    const int G = P->N2 / kColsPerBlock;
    if (obj && (st = get_objbuf(*P, iters, &sa.res, &sa.l1, s)) != CS_OK) return st;
    CS_LAUNCH(maybe_timed(timing, T_S_ISTA, s,
                          [&] { return launch_solve_dispatch(P->logN, 0, d / 2, obj != nullptr, sa, s); }));
    if (obj && (st = objective_reduce(sa.res, G, sa.l1, G, 0.5 / double(n / d), double(lambda), obj, iters, s)) != CS_OK)
      return st;
    return CS_OK;
  }
  if ((st = fill(reinterpret_cast<float*>(P->Y), size_t(P->N) * 2, 0.0f, s)) != CS_OK) return st;
  if ((st = fill(x, size_t(n), 0.0f, s)) != CS_OK) return st;
  double *res = nullptr, *l1 = nullptr;
  if (obj && (st = get_objbuf(*P, iters, &res, &l1, s)) != CS_OK) return st;
  const int nres = P->N1 / 2, nl1 = P->N2 / pass_b_cols(P->N1);
  PassAArgs a = argsA(*P);
  a.tau = tau;
  PassBArgs b = argsB(*P);
  b.thr = tau * lambda;
  b.u = x;
  // objective trace: obj[t-1] = F(x(t)); the row pass of iteration t + 1
  // sees x(t)'s spectrum, and one residual-only row pass follows the loop
  for (int t = 1; t <= iters; ++t) {
    a.res = (obj && t >= 2) ? res + size_t(t - 2) * nres : nullptr;
    CS_LAUNCH(maybe_timed(timing, T_A_ISTA, s, [&] { return launchA(*P, A_ISTA, a, s); }));
    b.last = (t == iters) && !obj;
    b.l1 = obj ? l1 + size_t(t - 1) * nl1 : nullptr;
    CS_LAUNCH(maybe_timed(timing, T_B_ISTA, s, [&] { return launchB(*P, B_ISTA, b, s); }));
  }
  if (obj) {
    a.res = res + size_t(iters - 1) * nres;
    CS_LAUNCH(launchA(*P, A_RES, a, s));
    if ((st = objective_reduce(res, nres, l1, nl1, 0.5 / double(n / d), double(lambda), obj, iters, s)) != CS_OK)
      return st;
  }
  return CS_OK;
}

}  // namespace
}  // namespace cs

using namespace cs;

extern "C" {

const char* cs_last_error(void) { return g_err.c_str(); }

int32_t cs_version(void) { return 100; }

size_t cs_unrolled_ckpt_bytes(int64_t n, int32_t d, int32_t Bt, int32_t K, int32_t every) {
  (void)d;
  if (n <= 0 || Bt <= 0 || K <= 0 || every <= 0) return 0;
  return size_t(ckpt_count(K, every)) * size_t(Bt) * size_t(n) * sizeof(float);
}

cs_status cs_unrolled_ista_fwd(const float* c, int64_t n, int32_t d, int32_t Bt, const float* y, const float* lam,
                               const float* tau, int32_t K, int32_t every, float* xK, void* ckpt,
                               cs_stream stream) {
  cs_status st = check_unrolled(c, n, d, Bt, y, lam, tau, K, every);
  if (st != CS_OK) return st;
  if (!xK) return fail(CS_EINVAL, "xK is NULL");
  if (ckpt_count(K, every) > 0 && !ckpt) return fail(CS_EINVAL, "ckpt is NULL");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  Plan* P = nullptr;
  if ((st = get_plan(n, d, &P)) != CS_OK) return st;
  UPlan* U = nullptr;
  if ((st = get_uplan(*P, Bt, every, K, &U)) != CS_OK) return st;
  const int64_t N = P->N, m = n / d;
  if ((st = setup_chat(*P, c, s)) != CS_OK) return st;
  // per-signal y_hat tables
  UStride us{};
  us.Y = N; us.yhat = N + 1; us.table = N + 1; us.in0 = m; us.u = n; us.out0 = m;
  us.rv = n; us.rd = n; us.xbar = n; us.vbar = n; us.part = P->N2 / ucol_cols(P->N1);
  {
    PassBArgs b = argsB(*P);
    b.Y = U->Y;
    b.in0 = y;
    CS_LAUNCH(launchUB(*P, B_FWD_UP, Bt, b, us, s));
    PassAArgs a = argsA(*P);
    a.Y = U->Y;
    a.table = U->yhat;
    CS_LAUNCH(launchUA(*P, A_SPEC, Bt, a, us, s));
  }
  if ((st = fill(reinterpret_cast<float*>(U->Y), size_t(Bt) * size_t(N) * 2, 0.0f, s)) != CS_OK) return st;
  if ((st = fill(xK, size_t(Bt) * size_t(n), 0.0f, s)) != CS_OK) return st;
  PassAArgs a = argsA(*P);
  a.Y = U->Y; a.yhat = U->yhat; a.tau_dev = tau;
  PassBArgs b = argsB(*P);
  b.Y = U->Y; b.u = xK; b.tau_dev = tau; b.lam_dev = lam;
  for (int t = 0; t < K; ++t) {
    a.t = t;
    CS_LAUNCH(launchUA(*P, A_ISTA, Bt, a, us, s));
    b.t = t;
    b.last = (t == K - 1);
    CS_LAUNCH(launchUB(*P, B_ISTA, Bt, b, us, s));
    if ((t + 1) % every == 0 && t + 1 < K) {
      float* dst = static_cast<float*>(ckpt) + size_t((t + 1) / every - 1) * size_t(Bt) * size_t(n);
      CS_HIP(hipMemcpyAsync(dst, xK, size_t(Bt) * size_t(n) * sizeof(float), hipMemcpyDeviceToDevice, s));
    }
  }
  g_err.clear();
  return CS_OK;
}

cs_status cs_unrolled_ista_bwd(const float* c, int64_t n, int32_t d, int32_t Bt, const float* y, const float* lam,
                               const float* tau, int32_t K, int32_t every, const void* ckpt, const float* g_xK,
                               float* g_lam, float* g_tau, float* g_y, cs_stream stream) {
  cs_status st = check_unrolled(c, n, d, Bt, y, lam, tau, K, every);
  if (st != CS_OK) return st;
  if (!g_xK || !g_lam || !g_tau || !g_y) return fail(CS_EINVAL, "a gradient pointer is NULL");
  if (ckpt_count(K, every) > 0 && !ckpt) return fail(CS_EINVAL, "ckpt is NULL");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  Plan* P = nullptr;
  if ((st = get_plan(n, d, &P)) != CS_OK) return st;
  UPlan* U = nullptr;
  if ((st = get_uplan(*P, Bt, every, K, &U)) != CS_OK) return st;
  const int64_t N = P->N, m = n / d;
  const int nblk = P->N2 / ucol_cols(P->N1);
  const size_t BN = size_t(Bt) * size_t(n);
  if ((st = setup_chat(*P, c, s)) != CS_OK) return st;
  UStride us{};
  us.Y = N; us.yhat = N + 1; us.ybar = N + 1; us.table = N + 1; us.in0 = 0; us.u = n; us.out0 = m;
  us.rv = n; us.rd = n; us.xbar = n; us.vbar = n; us.part = nblk;
  {
    UStride uy = us;
    uy.in0 = m;
    PassBArgs b = argsB(*P);
    b.Y = U->Y;
    b.in0 = y;
    CS_LAUNCH(launchUB(*P, B_FWD_UP, Bt, b, uy, s));
    PassAArgs a = argsA(*P);
    a.Y = U->Y;
    a.table = U->yhat;
    CS_LAUNCH(launchUA(*P, A_SPEC, Bt, a, us, s));
  }
  if ((st = fill(reinterpret_cast<float*>(U->ybar), size_t(Bt) * size_t(N + 1) * 2, 0.0f, s)) != CS_OK) return st;
  CS_HIP(hipMemcpyAsync(U->xbar, g_xK, BN * sizeof(float), hipMemcpyDeviceToDevice, s));
  const int nseg = (K + every - 1) / every;
  for (int sg = nseg - 1; sg >= 0; --sg) {
    const int t0 = sg * every, t1 = std::min(K, t0 + every);
    // x_{t0}: zero or the checkpoint; its spectrum into Y
    if (sg == 0) {
      if ((st = fill(U->xs, BN, 0.0f, s)) != CS_OK) return st;
    } else {
      const float* src = static_cast<const float*>(ckpt) + size_t(sg - 1) * BN;
      CS_HIP(hipMemcpyAsync(U->xs, src, BN * sizeof(float), hipMemcpyDeviceToDevice, s));
    }
    {
      UStride ux = us;
      ux.in0 = n;
      PassBArgs b = argsB(*P);
      b.Y = U->Y;
      b.in0 = U->xs;
      CS_LAUNCH(launchUB(*P, B_FWD_REAL, Bt, b, ux, s));
    }
    // recompute the segment, recording v_t and the step
    for (int t = t0; t < t1; ++t) {
      PassAArgs a = argsA(*P);
      a.Y = U->Y; a.yhat = U->yhat; a.tau_dev = tau; a.t = t;
      CS_LAUNCH(launchUA(*P, A_ISTA, Bt, a, us, s));
      PassBArgs b = argsB(*P);
      b.Y = U->Y; b.u = U->xs; b.tau_dev = tau; b.lam_dev = lam; b.t = t; b.last = (t == t1 - 1);
      b.rv = U->rv + size_t(t - t0) * BN;
      b.rd = U->rd + size_t(t - t0) * BN;
      CS_LAUNCH(launchUB(*P, B_ISTA_REC, Bt, b, us, s));
    }
    // reverse through the segment.  Step t's mask and sums (B_ADJ_V) read
    // xbar_t; inside the segment they are fused with step t+1's xbar update
    // (B_ADJ_XV), so xbar is stored only where a segment starts (B_ADJ_X),
    // for the step that follows the previous segment's recompute.
    auto adj_args = [&](int tt, PassBArgs& b) {
      b.tau_dev = tau; b.lam_dev = lam; b.t = tt;
      b.rv = U->rv + size_t(tt - t0) * BN;
      b.rd = U->rd + size_t(tt - t0) * BN;
      b.part = U->part + size_t(tt) * 2 * size_t(Bt) * size_t(nblk);
      b.part_q = Bt * nblk;
    };
    {
      PassBArgs b = argsB(*P);
      b.Y = U->Y; b.xbar = U->xbar; b.vbar = U->vbar;
      adj_args(t1 - 1, b);
      CS_LAUNCH(launchUB(*P, B_ADJ_V, Bt, b, us, s));
    }
    for (int t = t1 - 1; t >= t0; --t) {
      PassAArgs a = argsA(*P);
      a.Y = U->Y; a.ybar = U->ybar; a.tau_dev = tau; a.t = t;
      CS_LAUNCH(launchUA(*P, A_ADJ, Bt, a, us, s));
      PassBArgs bx = argsB(*P);
      bx.Y = U->Y; bx.vbar = U->vbar;
      if (t > t0) {
        adj_args(t - 1, bx);
        CS_LAUNCH(launchUB(*P, B_ADJ_XV, Bt, bx, us, s));
      } else {
        bx.xbar = U->xbar;
        CS_LAUNCH(launchUB(*P, B_ADJ_X, Bt, bx, us, s));
      }
    }
  }
  k_unrolled_grads<<<dim3(K), dim3(256), 0, s>>>(U->part, Bt * nblk, tau, lam, g_lam, g_tau);
  CS_HIP(hipGetLastError());
  // ybar = IDFT_m of the accumulated spectrum: tile onto n bins, inverse, decimate
  {
    PassAArgs a = argsA(*P);
    a.Y = U->Y; a.ybar = U->ybar;
    CS_LAUNCH(launchUA(*P, A_TILE, Bt, a, us, s));
    PassBArgs b = argsB(*P);
    b.Y = U->Y; b.out0 = g_y;
    CS_LAUNCH(launchUB(*P, B_OUT_DEC, Bt, b, us, s));
  }
  g_err.clear();
  return CS_OK;
}

size_t cs_workspace_bytes(int64_t n, int32_t d, int32_t mode) {
  if (mode < 0 || mode > 2) return 0;
  if (!is_pow2(n) || n < kMinN || n > kMaxN || (d != 1 && d != 2 && d != 4 && d != 8 && d != 16)) return 0;
  Plan p;
  plan_layout(n, d, p);
  return p.bytes;
}

cs_status cs_set_workspace(void* ws, size_t bytes) {
  if (ws && (reinterpret_cast<uintptr_t>(ws) & 255))
    return fail(CS_EINVAL, "workspace %p must be 256-byte aligned", ws);
  if (ws && bytes < cs_workspace_bytes(kMinN, 16, 0))
    return fail(CS_EINVAL, "workspace of %zu bytes is below the smallest plan (%zu bytes)", bytes,
                cs_workspace_bytes(kMinN, 16, 0));
  int dev = 0;
  CS_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(CS_ENOTSUP, "device %d beyond the supported %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lk(g_mu);
  ExtBlock& b = g_ws[dev];
  b.ptr = ws;
  b.bytes = ws ? bytes : 0;
  b.tables_n = 0;
  b.cleared = false;
  g_err.clear();
  return CS_OK;
}

cs_status cs_set_solver_path(int32_t path) {
  if (path < 0 || path > 2) return fail(CS_EINVAL, "path=%d must be 0, 1 or 2", path);
  std::lock_guard<std::mutex> lk(g_mu);
  g_path = path;
  g_err.clear();
  return CS_OK;
}

cs_status cs_check_device(cs_stream stream) {
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  CS_HIP(hipStreamSynchronize(s));
  int dev = 0;
  CS_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_mu);
  // the error flag of one block: read, and cleared if set
  auto check = [&](unsigned* bar, const char* what) -> cs_status {
    unsigned flag = 0;
    CS_HIP(hipMemcpy(&flag, bar + kBarErr, sizeof flag, hipMemcpyDeviceToHost));
    if (flag) {
      const unsigned zero = 0;
      CS_HIP(hipMemcpy(bar + kBarErr, &zero, sizeof zero, hipMemcpyHostToDevice));
      return fail(CS_EHIP, "a grid barrier wait exceeded its bound (%s)", what);
    }
    return CS_OK;
  };
  cs_status st = CS_OK;
  for (auto& kv : g_plans) {
    Plan& P = *kv.second;
    if (P.dev != dev) continue;
    char what[64];
    snprintf(what, sizeof what, "n=%lld d=%d", (long long)P.n, P.d);
    if ((st = check(P.bar, what)) != CS_OK) return st;
  }
  if ((st = batch_check_flags(dev)) != CS_OK) return st;
  if (dev >= 0 && dev < kMaxDevices) {
    for (ExtBlock* b : ext_blocks(dev))
      if (b->ptr && b->cleared && (st = check(static_cast<unsigned*>(b->ptr), "caller-provided memory")) != CS_OK)
        return st;
  }
  g_err.clear();
  return CS_OK;
}

cs_status cs_timing_enable(int32_t on) {
  std::lock_guard<std::mutex> lk(g_tmu);
  g_timing = (on != 0);
  g_err.clear();
  return CS_OK;
}

cs_status cs_timing_read(const char* kernel, int64_t* launches, double* total_ms) {
  if (!kernel || !launches || !total_ms) return fail(CS_EINVAL, "NULL argument");
  int kind = -1;
  for (int k = 0; k < T_COUNT; ++k)
    if (std::strcmp(kernel, kTimedNames[k]) == 0) kind = k;
  if (kind < 0) return fail(CS_EINVAL, "unknown kernel name '%s'", kernel);
  std::lock_guard<std::mutex> lk(g_tmu);
  int64_t cnt = 0;
  double tot = 0.0;
  std::vector<TimedLaunch> keep;
  for (auto& t : g_timed) {
    if (t.kind != kind) {
      keep.push_back(t);
      continue;
    }
    hipError_t e = hipEventSynchronize(t.stop);
    if (e != hipSuccess) return fail(CS_EHIP, "hipEventSynchronize failed: %s", hipGetErrorString(e));
    float ms = 0.0f;
    e = hipEventElapsedTime(&ms, t.start, t.stop);
    if (e != hipSuccess) return fail(CS_EHIP, "hipEventElapsedTime failed: %s", hipGetErrorString(e));
    tot += ms;
    ++cnt;
    g_event_pool.push_back(t.start);
    g_event_pool.push_back(t.stop);
  }
  g_timed.swap(keep);
  *launches = cnt;
  *total_ms = tot;
  g_err.clear();
  return CS_OK;
}

cs_status cs_circ_apply(const float* c, int64_t n, int32_t d, const float* x, float* y,
                        cs_stream stream) {
  cs_status st = check_common(c, n, d);
  if (st != CS_OK) return st;
  if (!x || !y) return fail(CS_EINVAL, "x or y is NULL");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  Plan V;
  if ((st = plan_for_call(n, d, s, V, nullptr)) != CS_OK) return st;
  const Plan* P = &V;
  if ((st = setup_chat(*P, c, s)) != CS_OK) return st;
  PassBArgs b = argsB(*P);
  b.in0 = x;
  CS_LAUNCH(launchB(*P, B_FWD_REAL, b, s));
  CS_LAUNCH(launchA(*P, A_MUL, argsA(*P), s));
  b = argsB(*P);
  b.out0 = y;
  CS_LAUNCH(launchB(*P, B_OUT_DEC, b, s));
  g_err.clear();
  return CS_OK;
}

cs_status cs_circ_apply_T(const float* c, int64_t n, int32_t d, const float* r, float* x,
                          cs_stream stream) {
  cs_status st = check_common(c, n, d);
  if (st != CS_OK) return st;
  if (!r || !x) return fail(CS_EINVAL, "r or x is NULL");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  Plan V;
  if ((st = plan_for_call(n, d, s, V, nullptr)) != CS_OK) return st;
  const Plan* P = &V;
  if ((st = setup_chat(*P, c, s)) != CS_OK) return st;
  PassBArgs b = argsB(*P);
  b.in0 = r;
  CS_LAUNCH(launchB(*P, B_FWD_UP, b, s));
  CS_LAUNCH(launchA(*P, A_MULC, argsA(*P), s));
  b = argsB(*P);
  b.out0 = x;
  CS_LAUNCH(launchB(*P, B_OUT_ALL, b, s));
  g_err.clear();
  return CS_OK;
}

cs_status cs_circ_apply_direct(const float* c, int64_t n, int32_t d, const float* x, float* y,
                               cs_stream stream) {
  cs_status st = check_common(c, n, d);
  if (st != CS_OK) return st;
  if (d < 2) return fail(CS_EINVAL, "d=%d: the direct products take d in {2, 4, 8, 16}", d);
  if (n < 256) return fail(CS_EINVAL, "n=%lld: the direct products take n >= 256", (long long)n);
  if (!x || !y) return fail(CS_EINVAL, "x or y is NULL");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  CS_LAUNCH(timed(T_DIRECT, s, [&] { return launch_direct(0, d, c, x, y, n, s); }));
  g_err.clear();
  return CS_OK;
}

cs_status cs_circ_apply_T_direct(const float* c, int64_t n, int32_t d, const float* r, float* x,
                                 cs_stream stream) {
  cs_status st = check_common(c, n, d);
  if (st != CS_OK) return st;
  if (d < 2) return fail(CS_EINVAL, "d=%d: the direct products take d in {2, 4, 8, 16}", d);
  if (n < 256) return fail(CS_EINVAL, "n=%lld: the direct products take n >= 256", (long long)n);
  if (!r || !x) return fail(CS_EINVAL, "r or x is NULL");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  CS_LAUNCH(timed(T_DIRECT_T, s, [&] { return launch_direct(1, d, c, r, x, n, s); }));
  g_err.clear();
  return CS_OK;
}

cs_status cs_circ_norm_bound(const float* c, int64_t n, float* out, cs_stream stream) {
  cs_status st = check_common(c, n, 2);
  if (st != CS_OK) return st;
  if (!out) return fail(CS_EINVAL, "out is NULL");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  Plan V;
  if ((st = plan_for_call(n, 2, s, V, nullptr)) != CS_OK) return st;
  const Plan* P = &V;
  if ((st = setup_chat(*P, c, s)) != CS_OK) return st;
  if ((st = fill(out, 1, 0.0f, s)) != CS_OK) return st;
  if ((st = max_abs2(P->chat, P->N + 1, out, s)) != CS_OK) return st;
  g_err.clear();
  return CS_OK;
}

cs_status cs_box_blur_generator(const float* c, int64_t n, int32_t L, float* out, cs_stream stream) {
  cs_status st = check_common(c, n, 2);
  if (st != CS_OK) return st;
  if (!out) return fail(CS_EINVAL, "out is NULL");
  if (out == c) return fail(CS_EINVAL, "out must not alias c");
  if (L < 1 || L > 4096 || L > n) return fail(CS_EINVAL, "L=%d must be in [1, min(n, 4096)]", L);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const unsigned grid = unsigned(std::min<int64_t>((n + 255) / 256, 4096));
  k_box_blur<<<dim3(grid), dim3(256), 0, s>>>(c, n, L, out);
  CS_LAUNCH(hipGetLastError());
  g_err.clear();
  return CS_OK;
}

cs_status cs_ista_solve(const float* c, int64_t n, int32_t d, const float* y, float lambda,
                        float tau, int32_t iters, float* x, float* obj, cs_stream stream) {
  cs_status st = check_ista(c, n, d, y, lambda, tau, iters, x);
  if (st != CS_OK) return st;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (iters == 0) {
    if ((st = fill(x, size_t(n), 0.0f, s)) != CS_OK) return st;
    g_err.clear();
    return CS_OK;
  }
  Plan V;
  if ((st = plan_for_call(n, d, s, V, nullptr)) != CS_OK) return st;
  if ((st = ista_run(V, c, y, lambda, tau, iters, x, obj, s, true)) != CS_OK) return st;
  g_err.clear();
  return CS_OK;
}

cs_status cs_ista_solve_noalloc(const float* c, int64_t n, int32_t d, const float* y, float lambda, float tau,
                                int32_t iters, float* x, cs_stream stream) {
  cs_status st = check_ista(c, n, d, y, lambda, tau, iters, x);
  if (st != CS_OK) return st;
  if (n > kNoAllocMaxN)
    return fail(CS_EINVAL, "n=%lld exceeds the allocation-free limit n <= %lld", (long long)n,
                (long long)kNoAllocMaxN);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (iters == 0) {
    if ((st = fill(x, size_t(n), 0.0f, s)) != CS_OK) return st;
    g_err.clear();
    return CS_OK;
  }
  int dev = 0;
  CS_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(CS_ENOTSUP, "device %d beyond the supported %d", dev, kMaxDevices);
  Plan V;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    ExtBlock& blk = g_noalloc[dev];
    if (!blk.ptr) {
      // once per device, with that device current: the device address of
      // this device's copy of `scratch`
      void* ptr = nullptr;
      const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !ptr)
        return fail(CS_EHIP, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
      blk.ptr = ptr;
      blk.bytes = sizeof(scratch);
      blk.tables_n = 0;
      blk.cleared = false;
    }
    if ((st = bind_external(dev, n, d, blk, s, V)) != CS_OK) return st;
  }
  if ((st = ista_run(V, c, y, lambda, tau, iters, x, nullptr, s, false)) != CS_OK) return st;
  g_err.clear();
  return CS_OK;
}

cs_status cs_cpadmm_solve(const float* c, int64_t n, const int64_t* omega_host, int64_t m, const float* y,
                          float alpha, float rho, float sigma, float tau, int32_t iters, float* x, float* v,
                          float* z, float* mu, float* nu, cs_stream stream) {
  if (!c || !y || !x || !v || !z || !mu || !nu) return fail(CS_EINVAL, "a device array is NULL");
  if (!is_pow2(n) || n < kCpMinN || n > kCpMaxN)
    return fail(CS_EINVAL, "n=%lld must be a power of two in [%lld, %lld]", (long long)n, (long long)kCpMinN,
                (long long)kCpMaxN);
  if (m < 1 || m > n) return fail(CS_EINVAL, "m=%lld must be in [1, n]", (long long)m);
  if (!omega_host) return fail(CS_EINVAL, "omega is NULL");
  if (!finite(alpha) || alpha < 0.0f) return fail(CS_EINVAL, "alpha=%g must be finite and >= 0", alpha);
  if (!finite(rho) || rho <= 0.0f) return fail(CS_EINVAL, "rho=%g must be finite and > 0", rho);
  if (!finite(sigma) || sigma <= 0.0f) return fail(CS_EINVAL, "sigma=%g must be finite and > 0", sigma);
  if (!finite(tau) || tau <= 0.0f) return fail(CS_EINVAL, "tau=%g must be finite and > 0", tau);
  if (iters < 0) return fail(CS_EINVAL, "iters=%d must be >= 0", iters);
  // Omega: distinct indices in [0, n), in any order
  std::vector<int> idx(static_cast<size_t>(m));
  {
    std::vector<int64_t> sorted(omega_host, omega_host + m);
    std::sort(sorted.begin(), sorted.end());
    if (sorted.front() < 0 || sorted.back() >= n)
      return fail(CS_EINVAL, "omega holds an index outside [0, n)");
    if (std::adjacent_find(sorted.begin(), sorted.end()) != sorted.end())
      return fail(CS_EINVAL, "omega holds a repeated index");
    for (int64_t i = 0; i < m; ++i) idx[size_t(i)] = int(omega_host[i]);
  }
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  cs_status st = CS_OK;
  for (float* p : {x, v, z, mu, nu})
    if ((st = fill(p, size_t(n), 0.0f, s)) != CS_OK) return st;
  if (iters == 0) {
    g_err.clear();
    return CS_OK;
  }
  Plan V;
  if ((st = plan_for_call(n, 2, s, V, nullptr)) != CS_OK) return st;
  if ((st = setup_chat(V, c, s)) != CS_OK) return st;
  // Omega's indices go to the device through the caller's x array (n floats
  // >= m ints), which the solve writes only at its end; the copy is waited
  // for before the host vector goes away.
  float2* W = nullptr;
  if ((st = get_cpbuf(V, &W, s)) != CS_OK) return st;
  // W: Yab (n complex), then mu_b, nu_b, py_b, om_b (N pairs each); all
  // start at zero (a = v + mu = 0, b = z - nu = 0)
  if ((st = fill(reinterpret_cast<float*>(W), size_t(n) * 2 + 8 * size_t(V.N), 0.0f, s)) != CS_OK) return st;
  float2* mu_b = W + n;
  float2* nu_b = mu_b + V.N;
  float2* py_b = nu_b + V.N;
  float2* om_b = py_b + V.N;
  int* didx = reinterpret_cast<int*>(x);
  CS_HIP(hipMemcpyAsync(didx, idx.data(), idx.size() * sizeof(int), hipMemcpyHostToDevice, s));
  k_cp_scatter<<<dim3(unsigned(std::min<int64_t>((m + 255) / 256, 1024))), dim3(256), 0, s>>>(
      didx, m, y, V.N1, V.N2, cp_cb(V.N1), reinterpret_cast<float*>(py_b), reinterpret_cast<float*>(om_b));
  CS_HIP(hipGetLastError());
  CS_HIP(hipStreamSynchronize(s));
  CpArgs a{};
  a.Yab = W;
  a.mu_b = mu_b;
  a.nu_b = nu_b;
  a.py_b = py_b;
  a.om_b = om_b;
  a.chat = V.chat;
  a.twk1 = V.twk1;
  a.twp = V.twp;
  a.twlo = V.twlo;
  a.twhi = V.twhi;
  a.tw1 = V.tw1;
  a.tw2 = V.tw2;
  a.lo_bits = V.lo_bits;
  a.N1 = V.N1;
  a.N2 = V.N2;
  a.N = V.N;
  a.inv_n = 1.0f / float(n);
  a.rho = rho;
  a.sigma = sigma;
  a.tau = tau;
  a.thr = alpha / sigma;
  a.d_in = 1.0f / (1.0f + rho);
  a.d_out = 1.0f / rho;
  a.mu = mu;
  a.nu = nu;
  a.v = v;
  a.z = z;
  a.x = x;
  for (int t = 1; t <= iters; ++t) {
    CS_LAUNCH(timed(T_CP_ROW, s, [&] { return launchCpRow(V, a, s); }));
    CS_LAUNCH(timed(T_CP_COL, s, [&] { return launchCpCol(V, t == iters, a, s); }));
  }
  g_err.clear();
  return CS_OK;
}

cs_status cs_admm_solve(const float* c, int64_t n, int32_t d, const float* y, float lambda,
                        float rho, int32_t iters, int32_t warm, float* x, float* z, float* u,
                        float* obj, cs_stream stream) {
  cs_status st = check_common(c, n, d);
  if (st != CS_OK) return st;
  if (!y || !x || !z || !u) return fail(CS_EINVAL, "y, x, z or u is NULL");
  if (!finite(lambda) || lambda < 0.0f) return fail(CS_EINVAL, "lambda=%g must be finite and >= 0", lambda);
  if (!finite(rho) || rho <= 0.0f) return fail(CS_EINVAL, "rho=%g must be finite and > 0", rho);
  if (iters < 0) return fail(CS_EINVAL, "iters=%d must be >= 0", iters);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (iters == 0) {
    if (!warm) {
      if ((st = fill(x, size_t(n), 0.0f, s)) != CS_OK) return st;
      if ((st = fill(z, size_t(n), 0.0f, s)) != CS_OK) return st;
      if ((st = fill(u, size_t(n), 0.0f, s)) != CS_OK) return st;
    }
    g_err.clear();
    return CS_OK;
  }
  Plan V;
  if ((st = plan_for_call(n, d, s, V, nullptr)) != CS_OK) return st;
  const Plan* P = &V;
  if ((st = setup_chat(*P, c, s)) != CS_OK) return st;
  if ((st = setup_yhat(*P, y, s)) != CS_OK) return st;
  bool pers = false;
  if ((st = use_persistent(*P, 1, obj != nullptr, &pers)) != CS_OK) return st;
  if (pers) {
    if ((st = fill(reinterpret_cast<float*>(P->bar), kBarErr, 0.0f, s)) != CS_OK) return st;
    SolveArgs sa = solve_args(*P);
    sa.x = x; sa.z = z; sa.u = u;
    sa.iters = iters;
    sa.warm = warm ? 1 : 0;
    sa.rho = rho;
    sa.inv_rho = float(1.0 / double(rho));
    sa.d_rho = float(double(d) * double(rho));
    sa.thr = float(double(lambda) / double(rho));
    const int G = P->N2 / kColsPerBlock;
    if (obj && (st = get_objbuf(*P, iters, &sa.res, &sa.l1, s)) != CS_OK) return st;
    CS_LAUNCH(timed(T_S_ADMM, s, [&] { return launch_solve_dispatch(P->logN, 1, d / 2, obj != nullptr, sa, s); }));
    if (obj && (st = objective_reduce(sa.res, G, sa.l1, G, 0.5 / double(n / d), double(lambda), obj, iters, s)) != CS_OK)
      return st;
    g_err.clear();
    return CS_OK;
  }
  if (warm) {
    PassBArgs b0 = argsB(*P);
    b0.in0 = z;
    b0.in1 = u;
    CS_LAUNCH(launchB(*P, B_FWD_ZMU, b0, s));
  } else {
    if ((st = fill(reinterpret_cast<float*>(P->Y), size_t(P->N) * 2, 0.0f, s)) != CS_OK) return st;
    if ((st = fill(u, size_t(n), 0.0f, s)) != CS_OK) return st;
  }
  PassAArgs a = argsA(*P);
  a.rho = rho;
  a.inv_rho = float(1.0 / double(rho));
  a.d_rho = float(double(d) * double(rho));
  PassBArgs b = argsB(*P);
  b.thr = float(double(lambda) / double(rho));
  b.out0 = x;
  b.out1 = z;
  b.u = u;
  double *res = nullptr, *l1 = nullptr;
  if (obj && (st = get_objbuf(*P, iters, &res, &l1, s)) != CS_OK) return st;
  const int nres = P->N1 / 2, nl1 = P->N2 / pass_b_cols(P->N1);
  // objective trace: obj[t-1] = F(x(t)), both parts from iteration t
  for (int t = 1; t <= iters; ++t) {
    a.res = obj ? res + size_t(t - 1) * nres : nullptr;
    CS_LAUNCH(timed(T_A_ADMM, s, [&] { return launchA(*P, A_ADMM, a, s); }));
    b.last = (t == iters);
    b.l1 = obj ? l1 + size_t(t - 1) * nl1 : nullptr;
    CS_LAUNCH(timed(T_B_ADMM, s, [&] { return launchB(*P, B_ADMM, b, s); }));
  }
  if (obj) {
    if ((st = objective_reduce(res, nres, l1, nl1, 0.5 / double(n / d), double(lambda), obj, iters, s)) != CS_OK)
      return st;
  }
  g_err.clear();
  return CS_OK;
}

}  // extern "C"
