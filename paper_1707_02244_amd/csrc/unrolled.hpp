// Row and column passes over a batch of equal-length signals (grid y =
// signal), used by the unrolled ISTA (signals sharing one sensing operator:
// forward with per-iteration parameters and a checkpointed reverse pass).
//
// The row and column passes of kernels.hpp run with a second grid dimension
// over the signals of the batch; each signal has its own spectrum buffer,
// y_hat table, state and records, found by per-signal strides (c_hat is
// shared).  The reverse pass is the adjoint of the recursion
//     v_t = x_{t-1} + tau_t A^T (y - A x_{t-1}),  x_t = eta_{tau_t lam_t}(v_t):
//     vbar_t = M_t xbar_t,  M_t = 1[|v_t| > tau_t lam_t]
//     d theta_t = -sum sgn(v_t) vbar_t,  lambar_t = tau_t d theta_t,
//     taubar_t = lam_t d theta_t + sum vbar_t g_t,
//     ybar += tau_t A vbar_t,  xbar_{t-1} = vbar_t - tau_t A^T A vbar_t.
// A vbar_t is accumulated in the m-point spectral domain (row pass A_ADJ) and
// brought back to the time domain once at the end (A_TILE + decimation).
#pragma once
#include "kernels.hpp"

namespace cs {

// Per-signal strides, in elements of each buffer's type (0: shared).
struct UStride {
  long long Y;      // row and column pass spectrum buffer (float2)
  long long yhat;   // y_hat table (float2)
  long long ybar;   // ybar spectrum (float2)
  long long table;  // A_SPEC destination (float2)
  long long in0;    // column-pass input (float)
  long long u;      // column-pass state (float)
  long long out0;   // column-pass output (float)
  long long rv, rd, xbar, vbar;   // records and adjoint state (float)
  long long part;   // partial sums (double): per signal, then + blockIdx.x
  long long chat;   // c_hat table (float2): 0 when the signals share c
  long long par;    // per-signal parameters tau_dev / lam_dev (float): 0 when
                    //   they are per iteration (indexed by t) instead
};

// Work per workgroup: about CS_U_ROW_PTS complex points per row item (AI
// consecutive row pairs) and CS_U_COL_PTS per column item (CB adjacent
// columns, at least 8), so that short signals do not run as many tiny
// workgroups.  N1 >= N2 / 4 for every plan, so AI <= N2 / 8 divides N1 / 2.
#ifndef CS_U_ROW_PTS
#define CS_U_ROW_PTS 2048
#endif
#ifndef CS_U_COL_PTS
#define CS_U_COL_PTS 2048
#endif
constexpr int urow_pairs(int N2) {
  const int ai = CS_U_ROW_PTS / (2 * N2);
  const int cap = N2 / 8 > 1 ? N2 / 8 : 1;
  return ai < 1 ? 1 : (ai > cap ? cap : ai);
}
// capped at 2 N1, the smaller of the two N2 a plan can have, so that it
// divides N2
constexpr int ucol_cols(int N1) {
  const int cb = CS_U_COL_PTS / N1;
  const int w = cb > 2 * N1 ? 2 * N1 : cb;
  return w < kColsPerBlock ? kColsPerBlock : w;
}

template <int N2, int OP, int D2>
__global__ __launch_bounds__(kThreads) void k_urow(PassAArgs a, UStride st) {
  constexpr int AI = urow_pairs(N2);
  constexpr int LD = N2 + kPadA;
  constexpr bool TW_LDS = (lds_rows(2 * AI * LD) + N2) * 8 <= 160 * 1024 - 1024;
  __shared__ float2 lds[lds_rows(2 * AI * LD)];
  __shared__ float2 tws_l[TW_LDS ? N2 : 1];
  const long long b = blockIdx.y;
  a.Y += b * st.Y;
  a.chat += b * st.chat;
  if (a.tau_dev) a.tau_dev += b * st.par;
  if (a.yhat) a.yhat += b * st.yhat;
  if (a.ybar) a.ybar += b * st.ybar;
  if (a.table) a.table += b * st.table;
  if constexpr (TW_LDS) {
    for (unsigned i = threadIdx.x; i < N2; i += kThreads) tws_l[i] = a.tw2[i];
  }
  __syncthreads();
  rowpass<N2, OP, D2, kThreads, false, AI>(a, blockIdx.x * AI, lds, TW_LDS ? tws_l : a.tw2, threadIdx.x);
}

template <int N1, int MODE>
__global__ __launch_bounds__(kThreads) void k_ucol(PassBArgs a, UStride st) {
  constexpr int CB = ucol_cols(N1);
  __shared__ float2 lds[lds_padded(N1 * CB)];
  __shared__ float2 tws[N1];
  const long long b = blockIdx.y;
  a.Y += b * st.Y;
  if (a.in0) a.in0 += b * st.in0;
  if (a.u) a.u += b * st.u;
  if (a.out0) a.out0 += b * st.out0;
  if (a.rv) a.rv += b * st.rv;
  if (a.rd) a.rd += b * st.rd;
  if (a.xbar) a.xbar += b * st.xbar;
  if (a.vbar) a.vbar += b * st.vbar;
  if (a.part) a.part += b * st.part + blockIdx.x;
  if (a.tau_dev) a.tau_dev += b * st.par;
  if (a.lam_dev) a.lam_dev += b * st.par;
  for (unsigned i = threadIdx.x; i < N1; i += kThreads) tws[i] = a.tw1[i];
  __syncthreads();
  colpass<N1, MODE, kThreads, false, CB>(a, blockIdx.x, lds, tws, threadIdx.x);
}

}  // namespace cs
