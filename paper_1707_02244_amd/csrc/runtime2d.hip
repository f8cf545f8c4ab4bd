// Host runtime and C ABI of the 2-D path (sensing with a blur, A = P C H on
// an R x C image, 2x2 decimation).
//
// A plan per (device, R, C) holds the twiddle tables (double precision,
// rounded to float) and the workspace: the transposed row-transformed
// spectrum T[k2][r] (H = C/2 packed columns of R complex values), the table
// of g_hat = DFT2(s) DFT2(h) at the bins the column pass visits
// ([H/2 + 1][2][R]) and the table of Y_hat = DFT2(y) ([H/2 + 1][R/2]).
#include <hip/hip_runtime.h>

#include <cstring>
#include <map>
#include <memory>
#include <tuple>
#include <vector>

#include "cscirc.h"
#include "kernels2d.hpp"
#include "launch.hpp"
#include "rt_common.hpp"

namespace cs {
namespace {
using namespace rt;

constexpr int kMinSide = 16;
constexpr int kMaxRows = 8192;
constexpr int kMaxCols = 4096;

struct Plan2D {
  int dev = 0;
  int R = 0, C = 0, H = 0;
  float2* mem = nullptr;
  float2 *T = nullptr, *G = nullptr, *Yt = nullptr;
  float2 *twR = nullptr, *twH = nullptr, *twc = nullptr;
  double* objbuf = nullptr;
  size_t obj_cap = 0;
  size_t g_count() const { return size_t(H / 2 + 1) * 2 * size_t(R); }
  size_t y_count() const { return size_t(H / 2 + 1) * size_t(R / 2); }
  int col_grid() const { return H / 2; }
  int row_grid() const { return R / kRows2; }
};

// Never destroyed (see the 1-D plan cache): no HIP call during static
// destruction; the device memory is returned with the process.
auto& g_plans2 = *new std::map<std::tuple<int, int, int>, std::unique_ptr<Plan2D>>();

cs_status get_plan2(int R, int C, Plan2D** out) {
  int dev = 0;
  CS_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_mu);
  auto key = std::make_tuple(dev, R, C);
  auto it = g_plans2.find(key);
  if (it != g_plans2.end()) {
    *out = it->second.get();
    return CS_OK;
  }
  auto p = std::make_unique<Plan2D>();
  p->dev = dev;
  p->R = R;
  p->C = C;
  p->H = C / 2;
  auto up = [](size_t v) { return (v + 63) & ~size_t(63); };
  const size_t oT = 0, oG = oT + up(size_t(p->H) * R), oY = oG + up(p->g_count());
  const size_t oTR = oY + up(p->y_count()), oTH = oTR + up(R), oTC = oTH + up(p->H);
  const size_t total = oTC + up(p->H / 2 + 1);
  hipError_t e = hipMalloc(&p->mem, total * sizeof(float2));
  if (e != hipSuccess)
    return fail(CS_ENOMEM, "hipMalloc of %zu bytes for the 2-D plan %dx%d failed: %s", total * sizeof(float2), R, C,
                hipGetErrorString(e));
  float2* b = p->mem;
  p->T = b + oT; p->G = b + oG; p->Yt = b + oY;
  p->twR = b + oTR; p->twH = b + oTH; p->twc = b + oTC;
  std::vector<float2> h(total - oTR);
  for (int i = 0; i < R; ++i) h[oTR - oTR + i] = root(i, R);
  for (int i = 0; i < p->H; ++i) h[oTH - oTR + i] = root(i, p->H);
  for (int i = 0; i <= p->H / 2; ++i) h[oTC - oTR + i] = root(i, C);
  e = hipMemcpy(b + oTR, h.data(), h.size() * sizeof(float2), hipMemcpyHostToDevice);
  if (e != hipSuccess) return fail(CS_EHIP, "hipMemcpy of 2-D plan tables failed: %s", hipGetErrorString(e));
  *out = p.get();
  g_plans2[key] = std::move(p);
  return CS_OK;
}

hipError_t launch_col(const Plan2D& P, int op, const Col2Args& a, hipStream_t s) {
  switch (P.R) {
#define CS_CASE(L) case L: return launch2_col<L>(op, P.col_grid(), a, s);
    CS_CASE(16) CS_CASE(32) CS_CASE(64) CS_CASE(128) CS_CASE(256) CS_CASE(512) CS_CASE(1024) CS_CASE(2048)
    CS_CASE(4096) CS_CASE(8192)
#undef CS_CASE
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_row(const Plan2D& P, int mode, const Row2Args& a, hipStream_t s) {
  switch (P.H) {
#define CS_CASE(L) case L: return launch2_row<L>(mode, P.row_grid(), a, s);
    CS_CASE(8) CS_CASE(16) CS_CASE(32) CS_CASE(64) CS_CASE(128) CS_CASE(256) CS_CASE(512) CS_CASE(1024)
    CS_CASE(2048)
#undef CS_CASE
    default: return hipErrorInvalidValue;
  }
}

Col2Args col_args(const Plan2D& P) {
  Col2Args a{};
  a.T = P.T; a.G = P.G; a.Yt = P.Yt; a.twR = P.twR; a.twc = P.twc;
  a.H = P.H;
  a.inv_n = float(1.0 / (double(P.R) * double(P.C)));
  return a;
}

Row2Args row_args(const Plan2D& P) {
  Row2Args a{};
  a.T = P.T; a.twH = P.twH; a.R = P.R; a.H = P.H;
  return a;
}

cs_status check2(const float* s, int R, int C) {
  if (!s) return fail(CS_EINVAL, "s is NULL");
  if (!is_pow2(R) || R < kMinSide || R > kMaxRows)
    return fail(CS_EINVAL, "rows=%d must be a power of two in [%d, %d]", R, kMinSide, kMaxRows);
  if (!is_pow2(C) || C < kMinSide || C > kMaxCols)
    return fail(CS_EINVAL, "cols=%d must be a power of two in [%d, %d]", C, kMinSide, kMaxCols);
  return CS_OK;
}

// g_hat table: DFT2(s), times DFT2(h) when a blur is given.
cs_status setup_g(const Plan2D& P, const float* s, const float* h, hipStream_t st) {
  Row2Args r = row_args(P);
  r.in0 = s;
  CS_LAUNCH(launch_row(P, R2_FWD_REAL, r, st));
  Col2Args c = col_args(P);
  c.table = P.G;
  CS_LAUNCH(launch_col(P, C2_SPEC, c, st));
  if (h) {
    r.in0 = h;
    CS_LAUNCH(launch_row(P, R2_FWD_REAL, r, st));
    CS_LAUNCH(launch_col(P, C2_SPECMUL, c, st));
  }
  return CS_OK;
}

// Y_hat table: the spectrum of P^T y, whose bins (k1, p), k1 < R/2, are y's
// (R/2 x C/2)-point DFT.
cs_status setup_y(const Plan2D& P, const float* y, hipStream_t st) {
  Row2Args r = row_args(P);
  r.in0 = y;
  CS_LAUNCH(launch_row(P, R2_FWD_UP, r, st));
  Col2Args c = col_args(P);
  c.table = P.Yt;
  CS_LAUNCH(launch_col(P, C2_YHAT, c, st));
  return CS_OK;
}

cs_status get_objbuf2(Plan2D& P, int iters, double** res, double** l1, hipStream_t s) {
  const size_t nres = size_t(P.col_grid()), nl1 = size_t(P.row_grid());
  const size_t need = size_t(iters) * (nres + nl1);
  std::lock_guard<std::mutex> lk(g_mu);
  if (P.obj_cap < need) {
    CS_HIP(hipStreamSynchronize(s));
    if (P.objbuf) CS_HIP(hipFree(P.objbuf));
    P.objbuf = nullptr;
    P.obj_cap = 0;
    hipError_t e = hipMalloc(&P.objbuf, need * sizeof(double));
    if (e != hipSuccess)
      return fail(CS_ENOMEM, "hipMalloc of %zu bytes for the objective trace failed", need * sizeof(double));
    P.obj_cap = need;
  }
  *res = P.objbuf;
  *l1 = P.objbuf + size_t(iters) * nres;
  return CS_OK;
}

}  // namespace
}  // namespace cs

using namespace cs;

extern "C" {

cs_status cs2_apply(const float* s, const float* h, int32_t rows, int32_t cols, const float* x, float* y,
                    cs_stream stream) {
  cs_status st = check2(s, rows, cols);
  if (st != CS_OK) return st;
  if (!x || !y) return fail(CS_EINVAL, "x or y is NULL");
  hipStream_t hs = reinterpret_cast<hipStream_t>(stream);
  Plan2D* P = nullptr;
  if ((st = get_plan2(rows, cols, &P)) != CS_OK) return st;
  if ((st = setup_g(*P, s, h, hs)) != CS_OK) return st;
  Row2Args r = row_args(*P);
  r.in0 = x;
  CS_LAUNCH(launch_row(*P, R2_FWD_REAL, r, hs));
  CS_LAUNCH(launch_col(*P, C2_MUL, col_args(*P), hs));
  r.out0 = y;
  CS_LAUNCH(launch_row(*P, R2_OUT_DEC, r, hs));
  return ok();
}

cs_status cs2_apply_T(const float* s, const float* h, int32_t rows, int32_t cols, const float* r, float* x,
                      cs_stream stream) {
  cs_status st = check2(s, rows, cols);
  if (st != CS_OK) return st;
  if (!r || !x) return fail(CS_EINVAL, "r or x is NULL");
  hipStream_t hs = reinterpret_cast<hipStream_t>(stream);
  Plan2D* P = nullptr;
  if ((st = get_plan2(rows, cols, &P)) != CS_OK) return st;
  if ((st = setup_g(*P, s, h, hs)) != CS_OK) return st;
  Row2Args ra = row_args(*P);
  ra.in0 = r;
  CS_LAUNCH(launch_row(*P, R2_FWD_UP, ra, hs));
  CS_LAUNCH(launch_col(*P, C2_MULC, col_args(*P), hs));
  ra.out0 = x;
  CS_LAUNCH(launch_row(*P, R2_OUT_ALL, ra, hs));
  return ok();
}

cs_status cs2_norm_bound(const float* s, const float* h, int32_t rows, int32_t cols, float* out,
                         cs_stream stream) {
  cs_status st = check2(s, rows, cols);
  if (st != CS_OK) return st;
  if (!out) return fail(CS_EINVAL, "out is NULL");
  hipStream_t hs = reinterpret_cast<hipStream_t>(stream);
  Plan2D* P = nullptr;
  if ((st = get_plan2(rows, cols, &P)) != CS_OK) return st;
  if ((st = setup_g(*P, s, h, hs)) != CS_OK) return st;
  if ((st = fill(out, 1, 0.0f, hs)) != CS_OK) return st;
  if ((st = max_abs2(P->G, int(P->g_count()), out, hs)) != CS_OK) return st;
  return ok();
}

cs_status cs2_ista_solve(const float* s, const float* h, int32_t rows, int32_t cols, const float* y, float lambda,
                         float tau, int32_t iters, float* x, float* obj, cs_stream stream) {
  cs_status st = check2(s, rows, cols);
  if (st != CS_OK) return st;
  if (!y || !x) return fail(CS_EINVAL, "y or x is NULL");
  if (!std::isfinite(lambda) || lambda < 0.0f) return fail(CS_EINVAL, "lambda=%g must be finite and >= 0", lambda);
  if (!std::isfinite(tau) || tau <= 0.0f) return fail(CS_EINVAL, "tau=%g must be finite and > 0", tau);
  if (iters < 0) return fail(CS_EINVAL, "iters=%d must be >= 0", iters);
  hipStream_t hs = reinterpret_cast<hipStream_t>(stream);
  const size_t n = size_t(rows) * size_t(cols);
  if ((st = fill(x, n, 0.0f, hs)) != CS_OK) return st;
  if (iters == 0) return ok();
  Plan2D* P = nullptr;
  if ((st = get_plan2(rows, cols, &P)) != CS_OK) return st;
  if ((st = setup_g(*P, s, h, hs)) != CS_OK) return st;
  if ((st = setup_y(*P, y, hs)) != CS_OK) return st;
  if ((st = fill(reinterpret_cast<float*>(P->T), size_t(P->H) * size_t(P->R) * 2, 0.0f, hs)) != CS_OK) return st;
  double *res = nullptr, *l1 = nullptr;
  if (obj && (st = get_objbuf2(*P, iters, &res, &l1, hs)) != CS_OK) return st;
  const int nres = P->col_grid(), nl1 = P->row_grid();
  Col2Args c = col_args(*P);
  c.tau = tau;
  Row2Args r = row_args(*P);
  r.u = x;
  r.thr = tau * lambda;
  // objective trace: obj[t-1] = F(x(t)); the column pass of iteration t + 1
  // sees x(t)'s spectrum, and one residual-only column pass ends the loop
  for (int t = 1; t <= iters; ++t) {
    c.res = (obj && t >= 2) ? res + size_t(t - 2) * nres : nullptr;
    CS_LAUNCH(timed(T_C2_ISTA, hs, [&] { return launch_col(*P, C2_ISTA, c, hs); }));
    r.last = (t == iters) && !obj;
    r.l1 = obj ? l1 + size_t(t - 1) * nl1 : nullptr;
    CS_LAUNCH(timed(T_R2_ISTA, hs, [&] { return launch_row(*P, R2_ISTA, r, hs); }));
  }
  if (obj) {
    c.res = res + size_t(iters - 1) * nres;
    CS_LAUNCH(launch_col(*P, C2_RES, c, hs));
    const double m = double(rows / 2) * double(cols / 2);
    if ((st = objective_reduce(res, nres, l1, nl1, 0.5 / m, double(lambda), obj, iters, hs)) != CS_OK) return st;
  }
  return ok();
}

cs_status cs2_admm_solve(const float* s, const float* h, int32_t rows, int32_t cols, const float* y, float lambda,
                         float rho, int32_t iters, int32_t warm, float* x, float* z, float* u, float* obj,
                         cs_stream stream) {
  cs_status st = check2(s, rows, cols);
  if (st != CS_OK) return st;
  if (!y || !x || !z || !u) return fail(CS_EINVAL, "y, x, z or u is NULL");
  if (!std::isfinite(lambda) || lambda < 0.0f) return fail(CS_EINVAL, "lambda=%g must be finite and >= 0", lambda);
  if (!std::isfinite(rho) || rho <= 0.0f) return fail(CS_EINVAL, "rho=%g must be finite and > 0", rho);
  if (iters < 0) return fail(CS_EINVAL, "iters=%d must be >= 0", iters);
  hipStream_t hs = reinterpret_cast<hipStream_t>(stream);
  const size_t n = size_t(rows) * size_t(cols);
  if (iters == 0) {
    if (!warm) {
      if ((st = fill(x, n, 0.0f, hs)) != CS_OK) return st;
      if ((st = fill(z, n, 0.0f, hs)) != CS_OK) return st;
      if ((st = fill(u, n, 0.0f, hs)) != CS_OK) return st;
    }
    return ok();
  }
  Plan2D* P = nullptr;
  if ((st = get_plan2(rows, cols, &P)) != CS_OK) return st;
  if ((st = setup_g(*P, s, h, hs)) != CS_OK) return st;
  if ((st = setup_y(*P, y, hs)) != CS_OK) return st;
  Row2Args r = row_args(*P);
  if (warm) {
    r.in0 = z;
    r.in1 = u;
    CS_LAUNCH(launch_row(*P, R2_FWD_ZMU, r, hs));
  } else {
    if ((st = fill(reinterpret_cast<float*>(P->T), size_t(P->H) * size_t(P->R) * 2, 0.0f, hs)) != CS_OK) return st;
    if ((st = fill(u, n, 0.0f, hs)) != CS_OK) return st;
  }
  double *res = nullptr, *l1 = nullptr;
  if (obj && (st = get_objbuf2(*P, iters, &res, &l1, hs)) != CS_OK) return st;
  const int nres = P->col_grid(), nl1 = P->row_grid();
  Col2Args c = col_args(*P);
  c.rho = rho;
  r.in0 = r.in1 = nullptr;
  r.u = u;
  r.out0 = x;
  r.out1 = z;
  r.thr = float(double(lambda) / double(rho));
  // objective trace: obj[t-1] = F(x(t)), both parts from iteration t
  for (int t = 1; t <= iters; ++t) {
    c.res = obj ? res + size_t(t - 1) * nres : nullptr;
    CS_LAUNCH(timed(T_C2_ADMM, hs, [&] { return launch_col(*P, C2_ADMM, c, hs); }));
    r.last = (t == iters);
    r.l1 = obj ? l1 + size_t(t - 1) * nl1 : nullptr;
    CS_LAUNCH(timed(T_R2_ADMM, hs, [&] { return launch_row(*P, R2_ADMM, r, hs); }));
  }
  if (obj) {
    const double m = double(rows / 2) * double(cols / 2);
    if ((st = objective_reduce(res, nres, l1, nl1, 0.5 / m, double(lambda), obj, iters, hs)) != CS_OK) return st;
  }
  return ok();
}

}  // extern "C"
