// Host runtime and C ABI of the batched solvers (ISTA, Alg. 1; ADMM, Alg. 2,
// over many independent signals of different lengths and decimations).
//
// A batch plan, cached per (device, algorithm, lengths, decimations,
// offsets), holds one device block with:
//   - the barrier area of the persistent launch (counters, error flag, leave
//     counter);
//   - the signal descriptors, the row / column items of the schedule and each
//     workgroup's item ranges and size class;
//   - twiddle tables per distinct length (double precision on the host,
//     rounded to float);
//   - per signal, the spectrum buffer Y and the c_hat / y_hat tables.
// The schedule (workgroups per CU, and how the workgroups are shared among
// the size classes) is chosen by a tuner that times the candidate schedules
// on the first call for a batch shape, and can be kept in a file named by
// CSCIRC_TUNE_CACHE.  The solve itself is one cooperative launch, recorded
// once per (plan, iterations, warm start) in a HIP graph and replayed with
// hipGraphLaunch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <list>
#include <memory>
#include <string>
#include <vector>

#include "cscirc.h"
#include "batch_persist.hpp"
#include "launch.hpp"
#include "rt_common.hpp"

namespace cs {
namespace {
using namespace rt;

constexpr int kMaxCachedPlans = 4;     // batch plans kept per process (least recently used dropped)
constexpr uint64_t kPBWaitMs = 20;     // bound of one barrier wait
constexpr int kTuneIters = 16;         // iterations of one tuner trial
constexpr int kPolicies = 2;           // cost models the tuner tries (see class_shares)

struct Key {
  int dev = 0, alg = 0;
  std::vector<int64_t> n, off_n, off_m;
  std::vector<int32_t> d;
  bool operator==(const Key& o) const {
    return dev == o.dev && alg == o.alg && n == o.n && d == o.d && off_n == o.off_n && off_m == o.off_m;
  }
};

struct Schedule {
  int wg_per_cu = 0;
  int policy = 0;
  int grid = 0;
};

struct BPlan {
  Key key;
  int cus = 0;
  int max_per_cu = 0;
  uint64_t max_ticks = 0;
  size_t n_rows = 0, n_cols = 0;   // item counts (independent of the schedule)
  int max_grid = 0;
  char* mem = nullptr;
  size_t bytes = 0;
  unsigned* bar = nullptr;
  PSig* sigs = nullptr;
  PItem* rows = nullptr;
  PItem* cols = nullptr;
  unsigned* row_off = nullptr;
  unsigned* col_off = nullptr;
  unsigned* wg_class = nullptr;
  std::vector<PSig> hsig;          // descriptors as on the device
  Schedule sched;                  // schedule uploaded to the device
  bool tuned = false;
  std::string tune_table;          // the tuner's trials as JSON
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int exec_iters = -1, exec_warm = -1;
  bool use_graph = true;           // false once recording a graph failed
};

// Plans are owned by this list (front = most recently used) and, like the
// single-signal plans, never destroyed at static destruction: the list is a
// heap object that is never deleted.  A plan pushed out of the list frees its
// memory then (hipFree waits for the device).
auto& g_bplans = *new std::list<std::unique_ptr<BPlan>>();
std::string g_last_info;           // schedule report of the last batched call
hipStream_t g_capture[64] = {};    // per-device stream for recording graphs

size_t up256(size_t v) { return (v + 255) & ~size_t(255); }

void release(BPlan& p) {
  if (p.exec) (void)hipGraphExecDestroy(p.exec);
  if (p.graph) (void)hipGraphDestroy(p.graph);
  if (p.mem) (void)hipFree(p.mem);
  p.exec = nullptr;
  p.graph = nullptr;
  p.mem = nullptr;
}

// ---------------------------------------------------------------------------
// Size classes and the schedule
struct Class {
  int L = 0, d2 = 0;
  std::vector<int> sig;            // signal indices of this class
  double cost = 0.0;
  size_t rows = 0, cols = 0;       // item counts
};

std::vector<Class> classes_of(const Key& k) {
  std::vector<Class> cls;
  for (size_t i = 0; i < k.n.size(); ++i) {
    const int L = ilog2(k.n[i] / 2), d2 = k.d[i] / 2;
    auto it = std::find_if(cls.begin(), cls.end(), [&](const Class& c) { return c.L == L && c.d2 == d2; });
    if (it == cls.end()) {
      cls.push_back(Class{});
      it = cls.end() - 1;
      it->L = L;
      it->d2 = d2;
    }
    it->sig.push_back(int(i));
    it->rows += size_t(pb_n1(L) / 2 / pb_ai(L));
    it->cols += size_t(pb_n2(L) / pb_cbw(L));
  }
  // largest lengths first (the order of the workgroup ranges)
  std::sort(cls.begin(), cls.end(), [](const Class& a, const Class& b) { return a.L != b.L ? a.L > b.L : a.d2 < b.d2; });
  return cls;
}

// Estimated cost of a class per iteration.  Policy 0: FFT work of both
// passes, 2 N (log2 N + 4) per signal (the 4 stands for the loads, stores and
// the update).  Policy 1: the number of items (every item covers about the
// same number of points and pays the same global round trip and set of
// barriers, which dominate at these sizes).
double class_cost(const Class& c, int policy) {
  if (policy == 1) return double(c.rows + c.cols);
  const double N = double(int64_t(1) << c.L);
  return double(c.sig.size()) * 2.0 * N * (double(c.L) + 4.0);
}

// Workgroups per class: proportional to the cost (largest remainder), at
// least one, at most the class's larger item count.
std::vector<int> class_shares(std::vector<Class>& cls, int G, int policy) {
  const int K = int(cls.size());
  double tot = 0.0;
  for (Class& c : cls) tot += (c.cost = class_cost(c, policy));
  std::vector<int> g(K, 1);
  std::vector<int> cap(K);
  int left = G - K;
  for (int k = 0; k < K; ++k) cap[k] = int(std::max(cls[k].rows, cls[k].cols));
  // hand out the remaining workgroups one by one to the class whose cost per
  // workgroup is largest (and that can still use one)
  while (left > 0) {
    int best = -1;
    double bv = -1.0;
    for (int k = 0; k < K; ++k) {
      if (g[k] >= cap[k]) continue;
      const double v = cls[k].cost / double(g[k]);
      if (v > bv) { bv = v; best = k; }
    }
    if (best < 0) break;
    ++g[best];
    --left;
  }
  (void)tot;
  return g;
}

// Build the host arrays of a schedule: items in workgroup order, offsets and
// each workgroup's class.  Returns the grid actually used (workgroups that a
// class cannot use are not launched).
int build_schedule(const Key& k, int G, int policy, std::vector<PItem>& rows, std::vector<PItem>& cols,
                   std::vector<unsigned>& roff, std::vector<unsigned>& coff, std::vector<unsigned>& wcls) {
  std::vector<Class> cls = classes_of(k);
  std::vector<int> share = class_shares(cls, G, policy);
  rows.clear();
  cols.clear();
  roff.assign(1, 0u);
  coff.assign(1, 0u);
  wcls.clear();
  for (size_t c = 0; c < cls.size(); ++c) {
    const Class& C = cls[c];
    const int N1 = pb_n1(C.L), N2 = pb_n2(C.L), AI = pb_ai(C.L), CBW = pb_cbw(C.L);
    std::vector<PItem> cr, cc;
    for (int s : C.sig) {
      for (int w = 0; w < N1 / 2; w += AI) cr.push_back(PItem{unsigned(s), unsigned(w)});
      for (int b = 0; b < N2 / CBW; ++b) cc.push_back(PItem{unsigned(s), unsigned(b)});
    }
    const int gk = share[c];
    for (int j = 0; j < gk; ++j) {
      const size_t r0 = cr.size() * size_t(j) / size_t(gk), r1 = cr.size() * size_t(j + 1) / size_t(gk);
      const size_t c0 = cc.size() * size_t(j) / size_t(gk), c1 = cc.size() * size_t(j + 1) / size_t(gk);
      rows.insert(rows.end(), cr.begin() + r0, cr.begin() + r1);
      cols.insert(cols.end(), cc.begin() + c0, cc.begin() + c1);
      roff.push_back(unsigned(rows.size()));
      coff.push_back(unsigned(cols.size()));
      wcls.push_back(unsigned(C.L) << 4 | unsigned(C.d2));
    }
  }
  return int(wcls.size());
}

// ---------------------------------------------------------------------------
// Tuner cache file: one JSON object per line,
//   {"key": "<shape key>", "wg_per_cu": W, "policy": P, "ms": T}
std::string shape_key(const BPlan& p) {
  // the schedule depends on the multiset of (n, d), the algorithm and the
  // device's CU count, not on where the signals sit in memory
  std::vector<std::pair<int64_t, int>> nd;
  for (size_t i = 0; i < p.key.n.size(); ++i) nd.push_back({p.key.n[i], p.key.d[i]});
  std::sort(nd.begin(), nd.end());
  uint64_t h = 1469598103934665603ull;
  auto mix = [&](uint64_t v) { for (int b = 0; b < 8; ++b) { h ^= (v >> (8 * b)) & 0xff; h *= 1099511628211ull; } };
  for (auto& e : nd) { mix(uint64_t(e.first)); mix(uint64_t(e.second)); }
  char buf[128];
  snprintf(buf, sizeof buf, "alg%d-count%zu-cu%d-%016llx", p.key.alg, nd.size(), p.cus, (unsigned long long)h);
  return buf;
}

bool cache_lookup(const std::string& key, Schedule& s) {
  const char* path = std::getenv("CSCIRC_TUNE_CACHE");
  if (!path || !*path) return false;
  FILE* f = std::fopen(path, "r");
  if (!f) return false;
  char line[512];
  bool found = false;
  const std::string pat = "\"key\": \"" + key + "\"";
  while (std::fgets(line, sizeof line, f)) {
    if (!std::strstr(line, pat.c_str())) continue;
    const char* w = std::strstr(line, "\"wg_per_cu\": ");
    const char* q = std::strstr(line, "\"policy\": ");
    if (w && q) {
      s.wg_per_cu = std::atoi(w + 13);
      s.policy = std::atoi(q + 10);
      found = s.wg_per_cu >= 1 && s.policy >= 0 && s.policy < kPolicies;
    }
  }
  std::fclose(f);
  return found;
}

void cache_store(const std::string& key, const Schedule& s, double ms) {
  const char* path = std::getenv("CSCIRC_TUNE_CACHE");
  if (!path || !*path) return;
  FILE* f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f, "{\"key\": \"%s\", \"wg_per_cu\": %d, \"policy\": %d, \"ms\": %.4f}\n", key.c_str(), s.wg_per_cu,
               s.policy, ms);
  std::fclose(f);
}

// ---------------------------------------------------------------------------
cs_status upload_schedule(BPlan& p, const Schedule& want, hipStream_t s) {
  std::vector<PItem> rows, cols;
  std::vector<unsigned> roff, coff, wcls;
  const int G = build_schedule(p.key, want.wg_per_cu * p.cus, want.policy, rows, cols, roff, coff, wcls);
  if (G < 1 || G > p.max_grid || rows.size() != p.n_rows || cols.size() != p.n_cols)
    return fail(CS_EHIP, "batched schedule construction failed");
  CS_HIP(hipStreamSynchronize(s));
  CS_HIP(hipMemcpy(p.rows, rows.data(), rows.size() * sizeof(PItem), hipMemcpyHostToDevice));
  CS_HIP(hipMemcpy(p.cols, cols.data(), cols.size() * sizeof(PItem), hipMemcpyHostToDevice));
  CS_HIP(hipMemcpy(p.row_off, roff.data(), roff.size() * sizeof(unsigned), hipMemcpyHostToDevice));
  CS_HIP(hipMemcpy(p.col_off, coff.data(), coff.size() * sizeof(unsigned), hipMemcpyHostToDevice));
  CS_HIP(hipMemcpy(p.wg_class, wcls.data(), wcls.size() * sizeof(unsigned), hipMemcpyHostToDevice));
  p.sched = want;
  p.sched.grid = G;
  // a recorded graph holds the old grid size
  if (p.exec) { (void)hipGraphExecDestroy(p.exec); p.exec = nullptr; }
  if (p.graph) { (void)hipGraphDestroy(p.graph); p.graph = nullptr; }
  p.exec_iters = p.exec_warm = -1;
  return CS_OK;
}

PBatchArgs launch_args(const BPlan& p, int iters, int warm) {
  PBatchArgs a{};
  a.sigs = p.sigs;
  a.rows = p.rows;
  a.cols = p.cols;
  a.row_off = p.row_off;
  a.col_off = p.col_off;
  a.wg_class = p.wg_class;
  a.bar = p.bar;
  a.err = reinterpret_cast<int*>(p.bar + kBarErr);
  a.max_ticks = p.max_ticks;
  a.iters = iters;
  a.warm = warm;
  return a;
}

const void* kernel_of(int alg) { return alg ? batch_persist_kernel<1>() : batch_persist_kernel<0>(); }

hipError_t launch_direct(const BPlan& p, int iters, int warm, hipStream_t s) {
  PBatchArgs a = launch_args(p, iters, warm);
  void* params[] = {&a};
  return hipLaunchCooperativeKernel(kernel_of(p.key.alg), dim3(p.sched.grid), dim3(kPBThreads), params, 0, s);
}

// Record the cooperative launch into a graph (stream capture on a stream of
// the library's own); false if the runtime cannot record it.
bool record_graph(BPlan& p, int iters, int warm) {
  const int dev = p.key.dev;
  if (!g_capture[dev] && hipStreamCreateWithFlags(&g_capture[dev], hipStreamNonBlocking) != hipSuccess) return false;
  hipStream_t cs_ = g_capture[dev];
  if (p.exec) { (void)hipGraphExecDestroy(p.exec); p.exec = nullptr; }
  if (p.graph) { (void)hipGraphDestroy(p.graph); p.graph = nullptr; }
  if (hipStreamBeginCapture(cs_, hipStreamCaptureModeThreadLocal) != hipSuccess) return false;
  const hipError_t le = launch_direct(p, iters, warm, cs_);
  hipGraph_t g = nullptr;
  const hipError_t ee = hipStreamEndCapture(cs_, &g);
  if (le != hipSuccess || ee != hipSuccess || !g) {
    if (g) (void)hipGraphDestroy(g);
    (void)hipGetLastError();
    return false;
  }
  hipGraphExec_t ex = nullptr;
  if (hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) != hipSuccess || !ex) {
    (void)hipGraphDestroy(g);
    (void)hipGetLastError();
    return false;
  }
  p.graph = g;
  p.exec = ex;
  p.exec_iters = iters;
  p.exec_warm = warm;
  return true;
}

struct CallPtrs {
  const float *c, *y, *lam, *par;
  float *x, *z, *u;
};
cs_status set_pointers(BPlan& p, const CallPtrs& cp, hipStream_t s);

// Time a few iterations of the solve under each candidate schedule and keep
// the fastest.  Runs once per plan, on the caller's stream, reading the
// caller's inputs; the trials write their iterates to a temporary block, so
// the caller's x, z, u (a warm start's inputs) are not touched.  Trials start
// cold.
cs_status tune(BPlan& p, const CallPtrs& caller, hipStream_t s) {
  const std::string key = shape_key(p);
  Schedule best;
  std::string table = "[";
  if (cache_lookup(key, best) && best.wg_per_cu <= p.max_per_cu) {
    cs_status st = upload_schedule(p, best, s);
    if (st != CS_OK) return st;
    table += "{\"from_cache\": true}]";
    p.tune_table = table;
    p.tuned = true;
    return CS_OK;
  }
  // temporary iterates: the caller's layout (max offset + length) for x, z, u
  size_t span = 0;
  for (size_t i = 0; i < p.key.n.size(); ++i) span = std::max(span, size_t(p.key.off_n[i] + p.key.n[i]));
  float* tmp = nullptr;
  hipError_t me = hipMalloc(reinterpret_cast<void**>(&tmp), 3 * span * sizeof(float));
  if (me != hipSuccess) return fail(CS_ENOMEM, "hipMalloc of %zu bytes for the tuner's iterates failed",
                                    3 * span * sizeof(float));
  struct Free { float* p; ~Free() { (void)hipFree(p); } } free_tmp{tmp};
  CallPtrs tp = caller;
  tp.x = tmp;
  tp.z = tmp + span;
  tp.u = tmp + 2 * span;
  cs_status st0 = set_pointers(p, tp, s);
  if (st0 != CS_OK) return st0;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  CS_HIP(hipEventCreate(&e0));
  CS_HIP(hipEventCreate(&e1));
  double best_ms = 1e30;
  bool first = true;
  for (int w = 1; w <= p.max_per_cu; ++w) {
    for (int pol = 0; pol < kPolicies; ++pol) {
      Schedule cand;
      cand.wg_per_cu = w;
      cand.policy = pol;
      cs_status st = upload_schedule(p, cand, s);
      if (st != CS_OK) { (void)hipEventDestroy(e0); (void)hipEventDestroy(e1); return st; }
      double ms = 1e30;
      for (int rep = 0; rep < 2; ++rep) {
        CS_HIP(hipEventRecord(e0, s));
        CS_LAUNCH(launch_direct(p, kTuneIters, 0, s));
        CS_HIP(hipEventRecord(e1, s));
        CS_HIP(hipEventSynchronize(e1));
        float t = 0.f;
        CS_HIP(hipEventElapsedTime(&t, e0, e1));
        ms = std::min(ms, double(t));
      }
      char buf[160];
      snprintf(buf, sizeof buf, "%s{\"wg_per_cu\": %d, \"policy\": %d, \"grid\": %d, \"ms_%d_iters\": %.4f}",
               first ? "" : ", ", w, pol, p.sched.grid, kTuneIters, ms);
      table += buf;
      first = false;
      if (ms < best_ms) { best_ms = ms; best = cand; }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  table += "]";
  cs_status st = upload_schedule(p, best, s);
  if (st != CS_OK) return st;
  CS_HIP(hipStreamSynchronize(s));   // the trials are done before the block is freed
  cache_store(key, best, best_ms);
  p.tune_table = table;
  p.tuned = true;
  return set_pointers(p, caller, s);
}

// ---------------------------------------------------------------------------
cs_status get_bplan(const Key& k, BPlan** out) {
  for (auto it = g_bplans.begin(); it != g_bplans.end(); ++it) {
    if ((*it)->key == k) {
      g_bplans.splice(g_bplans.begin(), g_bplans, it);
      *out = g_bplans.front().get();
      return CS_OK;
    }
  }
  auto p = std::make_unique<BPlan>();
  p->key = k;
  CS_HIP(hipDeviceGetAttribute(&p->cus, hipDeviceAttributeMultiprocessorCount, k.dev));
  int khz = 0;
  if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, k.dev) != hipSuccess || khz <= 0) khz = 100000;
  p->max_ticks = uint64_t(khz) * kPBWaitMs;
  p->max_per_cu = k.alg ? batch_persist_blocks_per_cu<1>() : batch_persist_blocks_per_cu<0>();
  if (p->max_per_cu < 1) return fail(CS_EHIP, "the batched kernel cannot be resident on this device");
  p->max_grid = p->max_per_cu * p->cus;
  const size_t count = k.n.size();
  std::vector<int> lens;   // distinct log2 N
  for (size_t i = 0; i < count; ++i) {
    const int L = ilog2(k.n[i] / 2);
    if (std::find(lens.begin(), lens.end(), L) == lens.end()) lens.push_back(L);
    p->n_rows += size_t(pb_n1(L) / 2 / pb_ai(L));
    p->n_cols += size_t(pb_n2(L) / pb_cbw(L));
  }
  // layout of the block
  size_t off = 0;
  auto take = [&](size_t b) { const size_t r = off; off += up256(b); return r; };
  const size_t o_bar = take(size_t(kPBBarWords) * sizeof(unsigned));
  const size_t o_sig = take(count * sizeof(PSig));
  const size_t o_rows = take(p->n_rows * sizeof(PItem));
  const size_t o_cols = take(p->n_cols * sizeof(PItem));
  const size_t o_roff = take(size_t(p->max_grid + 1) * sizeof(unsigned));
  const size_t o_coff = take(size_t(p->max_grid + 1) * sizeof(unsigned));
  const size_t o_cls = take(size_t(p->max_grid) * sizeof(unsigned));
  struct Tw { int L; size_t t1, t2, lo, hi, k1, pp; };
  std::vector<Tw> tws;
  for (int L : lens) {
    const int N1 = pb_n1(L), N2 = pb_n2(L), lo = (L + 1) / 2;
    Tw t{L, 0, 0, 0, 0, 0, 0};
    t.t1 = take(size_t(N1) * 8);
    t.t2 = take(size_t(N2) * 8);
    t.lo = take((size_t(1) << lo) * 8);
    t.hi = take((size_t(1) << (L - lo)) * 8);
    t.k1 = take(size_t(N1) * 8);
    t.pp = take(size_t(N2) * 8);
    tws.push_back(t);
  }
  std::vector<size_t> o_scr(count);
  for (size_t i = 0; i < count; ++i) {
    const size_t N = size_t(k.n[i] / 2);
    o_scr[i] = take((N + 2 * (N + 1) + 64) * sizeof(float2));
  }
  p->bytes = off;
  hipError_t e = hipMalloc(reinterpret_cast<void**>(&p->mem), p->bytes);
  if (e != hipSuccess) return fail(CS_ENOMEM, "hipMalloc of %zu bytes for a batch plan failed", p->bytes);
  p->bar = reinterpret_cast<unsigned*>(p->mem + o_bar);
  p->sigs = reinterpret_cast<PSig*>(p->mem + o_sig);
  p->rows = reinterpret_cast<PItem*>(p->mem + o_rows);
  p->cols = reinterpret_cast<PItem*>(p->mem + o_cols);
  p->row_off = reinterpret_cast<unsigned*>(p->mem + o_roff);
  p->col_off = reinterpret_cast<unsigned*>(p->mem + o_coff);
  p->wg_class = reinterpret_cast<unsigned*>(p->mem + o_cls);
  // barrier area zero, twiddle tables from the host
  std::vector<unsigned> zero(kPBBarWords, 0u);
  CS_HIP(hipMemcpy(p->bar, zero.data(), zero.size() * sizeof(unsigned), hipMemcpyHostToDevice));
  for (const Tw& t : tws) {
    const int L = t.L, N1 = pb_n1(L), N2 = pb_n2(L), lo = (L + 1) / 2;
    const int64_t N = int64_t(1) << L, n = 2 * N, nlo = int64_t(1) << lo, nhi = N >> lo;
    auto put = [&](size_t o, int64_t cnt, auto fn) -> cs_status {
      std::vector<float2> h(static_cast<size_t>(cnt));
      for (int64_t i = 0; i < cnt; ++i) h[size_t(i)] = fn(i);
      CS_HIP(hipMemcpy(p->mem + o, h.data(), h.size() * sizeof(float2), hipMemcpyHostToDevice));
      return CS_OK;
    };
    cs_status st = CS_OK;
    if ((st = put(t.t1, N1, [&](int64_t i) { return root(i, N1); })) != CS_OK) return st;
    if ((st = put(t.t2, N2, [&](int64_t i) { return root(i, N2); })) != CS_OK) return st;
    if ((st = put(t.lo, nlo, [&](int64_t i) { return root(i, N); })) != CS_OK) return st;
    if ((st = put(t.hi, nhi, [&](int64_t i) { return root(i * nlo, N); })) != CS_OK) return st;
    if ((st = put(t.k1, N1, [&](int64_t i) { return root(i, n); })) != CS_OK) return st;
    if ((st = put(t.pp, N2, [&](int64_t i) { return root(i, 2 * int64_t(N2)); })) != CS_OK) return st;
  }
  // descriptors without the caller's pointers (filled per call)
  p->hsig.assign(count, PSig{});
  for (size_t i = 0; i < count; ++i) {
    PSig& g = p->hsig[i];
    std::memset(&g, 0, sizeof g);
    const int L = ilog2(k.n[i] / 2);
    const Tw& t = *std::find_if(tws.begin(), tws.end(), [&](const Tw& w) { return w.L == L; });
    float2* base = reinterpret_cast<float2*>(p->mem + o_scr[i]);
    const size_t N = size_t(k.n[i] / 2);
    g.Y = base;
    g.chat = base + N;
    g.yhat = base + 2 * N + 1;
    g.tw1 = reinterpret_cast<const float2*>(p->mem + t.t1);
    g.tw2 = reinterpret_cast<const float2*>(p->mem + t.t2);
    g.twlo = reinterpret_cast<const float2*>(p->mem + t.lo);
    g.twhi = reinterpret_cast<const float2*>(p->mem + t.hi);
    g.twk1 = reinterpret_cast<const float2*>(p->mem + t.k1);
    g.twp = reinterpret_cast<const float2*>(p->mem + t.pp);
    g.logN = L;
    g.lo_bits = (L + 1) / 2;
    g.d = k.d[i];
  }
  // the device descriptors are written by the first call (pointers differ)
  g_bplans.push_front(std::move(p));
  while (int(g_bplans.size()) > kMaxCachedPlans) {
    release(*g_bplans.back());
    g_bplans.pop_back();
  }
  *out = g_bplans.front().get();
  return CS_OK;
}

// Bring the device descriptors up to date with this call's pointers.
cs_status set_pointers(BPlan& p, const CallPtrs& cp, hipStream_t s) {
  std::vector<PSig> want = p.hsig;
  for (size_t i = 0; i < want.size(); ++i) {
    PSig& g = want[i];
    g.c = cp.c + p.key.off_n[i];
    g.y = cp.y + p.key.off_m[i];
    g.x = cp.x + p.key.off_n[i];
    g.z = cp.z ? cp.z + p.key.off_n[i] : nullptr;
    g.u = cp.u ? cp.u + p.key.off_n[i] : nullptr;
    g.lam = cp.lam + i;
    g.par = cp.par + i;
  }
  static_assert(sizeof(PSig) % 8 == 0, "");
  if (std::memcmp(want.data(), p.hsig.data(), want.size() * sizeof(PSig)) != 0) {
    CS_HIP(hipStreamSynchronize(s));
    CS_HIP(hipMemcpy(p.sigs, want.data(), want.size() * sizeof(PSig), hipMemcpyHostToDevice));
    p.hsig = want;
  }
  return CS_OK;
}

cs_status check_batch(int count, const int64_t* n, const int32_t* d, const int64_t* off_n, const int64_t* off_m) {
  if (count < 0) return fail(CS_EINVAL, "count=%d must be >= 0", count);
  if (count == 0) return CS_OK;
  if (!n || !d || !off_n || !off_m) return fail(CS_EINVAL, "a size, decimation or offset array is NULL");
  std::vector<std::pair<int64_t, int64_t>> span(static_cast<size_t>(count));
  for (int i = 0; i < count; ++i) {
    if (!is_pow2(n[i]) || n[i] < (int64_t(2) << kPBMinLogN) || n[i] > (int64_t(2) << kPBMaxLogN))
      return fail(CS_EINVAL, "n[%d]=%lld must be a power of two in [2^%d, 2^%d]", i, (long long)n[i],
                  kPBMinLogN + 1, kPBMaxLogN + 1);
    if (d[i] != 2 && d[i] != 4 && d[i] != 8) return fail(CS_EINVAL, "d[%d]=%d must be 2, 4 or 8", i, d[i]);
    if (off_n[i] < 0 || (off_n[i] & 1) || off_m[i] < 0)
      return fail(CS_EINVAL, "offsets of signal %d must be >= 0 (off_n even)", i);
    span[size_t(i)] = {off_n[i], off_n[i] + n[i]};
  }
  std::sort(span.begin(), span.end());
  for (size_t i = 1; i < span.size(); ++i)
    if (span[i].first < span[i - 1].second) return fail(CS_EINVAL, "the signals' n-length slices overlap");
  return CS_OK;
}

__global__ void k_zero_slices(const PSig* sigs, int count, int which) {
  const int s = blockIdx.y;
  if (s >= count) return;
  const PSig g = sigs[s];
  float* p = which == 0 ? g.x : (which == 1 ? g.z : g.u);
  const int64_t n = int64_t(2) << g.logN;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    p[i] = 0.0f;
}

cs_status batched(int alg, int32_t count, const int64_t* n_host, const int32_t* d_host, const int64_t* off_n,
                  const int64_t* off_m, const CallPtrs& cp, int iters, int warm, hipStream_t s) {
  Key k;
  CS_HIP(hipGetDevice(&k.dev));
  if (k.dev < 0 || k.dev >= 64) return fail(CS_ENOTSUP, "device %d beyond the supported range", k.dev);
  k.alg = alg;
  k.n.assign(n_host, n_host + count);
  k.d.assign(d_host, d_host + count);
  k.off_n.assign(off_n, off_n + count);
  k.off_m.assign(off_m, off_m + count);
  std::lock_guard<std::mutex> lk(g_mu);
  BPlan* p = nullptr;
  cs_status st = get_bplan(k, &p);
  if (st != CS_OK) return st;
  if ((st = set_pointers(*p, cp, s)) != CS_OK) return st;
  if (iters == 0) {
    // x(0) = 0 (ISTA); x = z = u = 0 (cold ADMM); a warm ADMM keeps its input
    if (alg == 0 || !warm) {
      const dim3 grid(64, unsigned(count));
      for (int which = 0; which < (alg == 0 ? 1 : 3); ++which) {
        k_zero_slices<<<grid, dim3(256), 0, s>>>(p->sigs, count, which);
        CS_HIP(hipGetLastError());
      }
    }
    g_err.clear();
    return CS_OK;
  }
  if (!p->tuned && (st = tune(*p, cp, s)) != CS_OK) return st;
  bool graphed = false;
  if (p->use_graph) {
    if (!p->exec || p->exec_iters != iters || p->exec_warm != warm) p->use_graph = record_graph(*p, iters, warm);
    if (p->use_graph) {
      hipGraphExec_t ex = p->exec;
      CS_LAUNCH(timed(T_BATCH, s, [&] { return hipGraphLaunch(ex, s); }));
      graphed = true;
    }
  }
  if (!graphed) CS_LAUNCH(timed(T_BATCH, s, [&] { return launch_direct(*p, iters, warm, s); }));
  char buf[256];
  snprintf(buf, sizeof buf,
           "{\"grid\": %d, \"wg_per_cu\": %d, \"policy\": %d, \"graph\": %s, \"key\": \"%s\", \"trials\": ",
           p->sched.grid, p->sched.wg_per_cu, p->sched.policy, graphed ? "true" : "false", shape_key(*p).c_str());
  g_last_info = std::string(buf) + p->tune_table + "}";
  g_err.clear();
  return CS_OK;
}

}  // namespace

namespace rt {
// Error flags of the batch plans on device `dev` (read and cleared); called
// by cs_check_device after the stream has been synchronised.
cs_status batch_check_flags(int dev) {
  for (auto& p : g_bplans) {
    if (p->key.dev != dev || !p->bar) continue;
    unsigned flag = 0;
    CS_HIP(hipMemcpy(&flag, p->bar + kBarErr, sizeof flag, hipMemcpyDeviceToHost));
    if (flag) {
      const unsigned zero = 0;
      CS_HIP(hipMemcpy(p->bar + kBarErr, &zero, sizeof zero, hipMemcpyHostToDevice));
      return fail(CS_EHIP, "a grid barrier wait of a batched solve exceeded its bound");
    }
  }
  return CS_OK;
}
}  // namespace rt
}  // namespace cs

using namespace cs;

extern "C" {

cs_status cs_ista_solve_batched(int32_t count, const int64_t* n_host, const int32_t* d_host,
                                const int64_t* off_n_host, const int64_t* off_m_host, const float* c_cat,
                                const float* y_cat, const float* lambda_dev, const float* tau_dev, int32_t iters,
                                float* x_cat, cs_stream stream) {
  cs_status st = check_batch(count, n_host, d_host, off_n_host, off_m_host);
  if (st != CS_OK) return st;
  if (count == 0) return ok();
  if (!c_cat || !y_cat || !lambda_dev || !tau_dev || !x_cat) return fail(CS_EINVAL, "a device array is NULL");
  if (iters < 0) return fail(CS_EINVAL, "iters=%d must be >= 0", iters);
  CallPtrs cp{c_cat, y_cat, lambda_dev, tau_dev, x_cat, nullptr, nullptr};
  return batched(0, count, n_host, d_host, off_n_host, off_m_host, cp, iters, 0,
                 reinterpret_cast<hipStream_t>(stream));
}

cs_status cs_admm_solve_batched(int32_t count, const int64_t* n_host, const int32_t* d_host,
                                const int64_t* off_n_host, const int64_t* off_m_host, const float* c_cat,
                                const float* y_cat, const float* lambda_dev, const float* rho_dev, int32_t iters,
                                int32_t warm, float* x_cat, float* z_cat, float* u_cat, cs_stream stream) {
  cs_status st = check_batch(count, n_host, d_host, off_n_host, off_m_host);
  if (st != CS_OK) return st;
  if (count == 0) return ok();
  if (!c_cat || !y_cat || !lambda_dev || !rho_dev || !x_cat || !z_cat || !u_cat)
    return fail(CS_EINVAL, "a device array is NULL");
  if (iters < 0) return fail(CS_EINVAL, "iters=%d must be >= 0", iters);
  CallPtrs cp{c_cat, y_cat, lambda_dev, rho_dev, x_cat, z_cat, u_cat};
  return batched(1, count, n_host, d_host, off_n_host, off_m_host, cp, iters, warm ? 1 : 0,
                 reinterpret_cast<hipStream_t>(stream));
}

cs_status cs_batched_schedule(char* buf, size_t cap) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!buf || cap == 0) return fail(CS_EINVAL, "buffer is NULL or empty");
  if (g_last_info.size() + 1 > cap) return fail(CS_EINVAL, "buffer of %zu bytes is too small (%zu needed)", cap,
                                                g_last_info.size() + 1);
  std::memcpy(buf, g_last_info.c_str(), g_last_info.size() + 1);
  return ok();
}

}  // extern "C"
