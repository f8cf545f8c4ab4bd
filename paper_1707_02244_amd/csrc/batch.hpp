// Batched ISTA over many independent signals of different lengths, in one
// launch.
//
// Each workgroup takes whole signals from a work queue (signals sorted by
// length, longest first, so the tail of the launch is short) and runs all
// iterations of ISTA (Alg. 1) on its signal alone.  Workgroups never wait
// for each other, so the launch cannot deadlock whatever the residency.  The
// per-signal arithmetic is the plain solver's: four-step N = N1 * N2 FFT of
// the packed real signal, the alias-class ISTA step in the frequency domain,
// the soft threshold (Eq. 4) on a time-domain iterate.  The signal's
// spectrum buffer, c_hat / y_hat tables and iterate live in global scratch
// (L2 / Infinity-Cache resident for all but the longest signals); a
// workgroup barrier separates the row and column passes.
//
// To keep enough memory traffic in flight per workgroup, each step of a
// pass handles 8192 complex points: AI row pairs at once in the row pass, CBB
// adjacent columns at once in the column pass.
#pragma once
#include "kernels.hpp"

namespace cs {

constexpr int kBThreads = 512;
constexpr int kBPoints = 8192;                       // complex points per step
constexpr int kBMinLogN = 9;                         // n = 2^10 ..
constexpr int kBMaxLogN = 17;                        // .. 2^18
constexpr int kBMaxN1 = 256;
constexpr int kBMaxN2 = 512;
constexpr int kBLds = lds_rows(kBPoints + 16 * kPadA) + 64;   // rows carry kPadA padding each

// Everything a workgroup needs for one signal (built on the host).
struct BatchSig {
  const float* c;          // generator, n
  const float* y;          // measurements, m
  float* x;                // iterate / output, n
  const float* lam;        // device scalar
  const float* tau;        // device scalar
  float2* Y;               // scratch: N complex
  float2* chat;            // scratch: N + 1 complex
  float2* yhat;            // scratch: N + 1 complex
  const float2* tw1;       // W_{N1}
  const float2* tw2;       // W_{N2}
  const float2* twlo;      // W_N^e, e < 2^lo_bits
  const float2* twhi;      // W_N^{e * 2^lo_bits}
  const float2* twk1;      // W_n^{k1}
  const float2* twp;       // W_{2 N2}^p
  int logN;                // N = 2^logN complex points
  int lo_bits;
  int pad[2];
};

// Row pass on AI consecutive row pairs starting at pair w0 (pair 0 is rows
// {0, N1/2}, pair w > 0 is rows {w, N1 - w}).  OP: A_SPEC (write X to
// `table`) or A_ISTA (the alias-class step, from the step's c_hat / y_hat).
template <int N1, int N2, int D2, int AI, int OP, int T>
__device__ __forceinline__ void batch_rows(const BatchSig& s, float2* table, int w0, bool zero_in,
                                           float tau, float2* __restrict__ lds,
                                           const float2* __restrict__ t2, unsigned tid) {
  constexpr int N = N1 * N2;
  constexpr int LDA = N2 + kPadA;
  constexpr int RA = 2 * AI;
  constexpr int EA = (RA * N2 + T - 1) / T;
  constexpr bool FA = (RA * N2) % T == 0;
  constexpr int M = N2 / D2;
  constexpr int NCLS = (OP == A_ISTA) ? AI * M + 1 : 1;
  constexpr int GPT = (NCLS + T - 1) / T;
  static_assert(lds_rows(RA * LDA) <= kBLds, "row step exceeds the LDS buffer");
  const int ng0 = (w0 == 0) ? (M + 1) : M;
  const int ncls = ng0 + (AI - 1) * M;
  auto row_of = [&](unsigned slot) -> unsigned {
    const unsigned w = w0 + (slot >> 1);
    return (slot & 1) ? (w ? N1 - w : (N1 >> 1)) : w;
  };
  struct Cls { int sa, sb, rowa, rowb, k2, mode; };
  auto decode = [&](unsigned q) -> Cls {
    const int pi = (q < (unsigned)ng0) ? 0 : 1 + (q - ng0) / M;
    const int lc = (q < (unsigned)ng0) ? q : (q - ng0) % M;
    const int w = w0 + pi;
    Cls c;
    if (w) { c.sa = 2 * pi; c.sb = 2 * pi + 1; c.rowa = w; c.rowb = N1 - w; c.k2 = lc; c.mode = 0; }
    else if (lc <= (M >> 1)) { c.sa = c.sb = 2 * pi; c.rowa = c.rowb = 0; c.k2 = lc; c.mode = 1; }
    else { c.sa = c.sb = 2 * pi + 1; c.rowa = c.rowb = N1 >> 1; c.k2 = lc - (M >> 1) - 1; c.mode = 2; }
    return c;
  };

  float2 gca[GPT][D2], gcb[GPT][D2], gy[GPT];
  {
    float2 rv[EA];
#pragma unroll
    for (int k = 0; k < EA; ++k) {
      const unsigned i = tid + k * T;
      if (FA || i < RA * N2) rv[k] = zero_in ? c2(0.f, 0.f) : s.Y[row_of(i / N2) * N2 + (i % N2)];
    }
    if constexpr (OP == A_ISTA) {
#pragma unroll
      for (int k = 0; k < GPT; ++k) {
        const unsigned q = tid + k * T;
        if (q < (unsigned)ncls) {
          const Cls c = decode(q);
#pragma unroll
          for (int l = 0; l < D2; ++l) {
            const int p = c.k2 + l * M;
            const int qq = (c.mode == 1) ? ((N2 - p) & (N2 - 1)) : (N2 - 1 - p);
            gca[k][l] = s.chat[c.rowa * N2 + p];
            gcb[k][l] = (c.mode == 1 && p == 0) ? s.chat[N] : s.chat[c.rowb * N2 + qq];
          }
          gy[k] = s.yhat[c.rowa * N2 + c.k2];
        }
      }
    }
#pragma unroll
    for (int k = 0; k < EA; ++k) {
      const unsigned i = tid + k * T;
      if (FA || i < RA * N2) lds[lpr((i / N2) * LDA + (i % N2))] = rv[k];
    }
  }
  __syncthreads();
  lds_fft<N2, RA, T, false, false, LDA>(lds, t2, tid);

  if constexpr (OP == A_SPEC) {
    // every position of every held row: X at that bin; the Nyquist bin from
    // row 0 position 0
    for (unsigned i = tid; i < RA * N2; i += T) {
      const unsigned slot = i / N2, p = i % N2;
      const unsigned row = row_of(slot);
      const unsigned w = w0 + (slot >> 1);
      unsigned qs, qp;   // partner slot / position of bin N - k
      if (w) { qs = slot ^ 1; qp = N2 - 1 - p; }
      else if ((slot & 1) == 0) { qs = slot; qp = (N2 - p) & (N2 - 1); }
      else { qs = slot; qp = N2 - 1 - p; }
      const float2 za = lds[lpr(slot * LDA + p)];
      const float2 zbc = cconj(lds[lpr(qs * LDA + qp)]);
      const float2 wt = cmul(s.twk1[row], s.twp[p]);
      const float2 P = cscale(cadd(za, zbc), 0.5f);
      const float2 Q = cscale(cmulmi(csub(za, zbc)), 0.5f);
      const float2 wq = cmul(wt, Q);
      table[row * N2 + p] = cadd(P, wq);
      if (row == 0 && p == 0) table[N] = cconj(csub(P, wq));
    }
    return;
  } else {
#pragma unroll
    for (int k = 0; k < GPT; ++k) {
      const unsigned q = tid + k * T;
      if (q >= (unsigned)ncls) continue;
      const Cls c = decode(q);
      const int sa = c.sa, sb = c.sb, k2 = c.k2, mode = c.mode;
      const bool write_b = !(mode == 1 && (k2 == 0 || k2 == (M >> 1)));
      const float2 wk1 = s.twk1[c.rowa];
      float2 Xa[D2], Xb[D2], gw[D2];
#pragma unroll
      for (int l = 0; l < D2; ++l) {
        const int p = k2 + l * M;
        const int qq = (mode == 1) ? ((N2 - p) & (N2 - 1)) : (N2 - 1 - p);
        gw[l] = cmul(wk1, s.twp[p]);
        const float2 za = lds[lpr(sa * LDA + p)];
        const float2 zbc = cconj(lds[lpr(sb * LDA + qq)]);
        const float2 P = cscale(cadd(za, zbc), 0.5f);
        const float2 Q = cscale(cmulmi(csub(za, zbc)), 0.5f);
        const float2 wq = cmul(gw[l], Q);
        Xa[l] = cadd(P, wq);
        Xb[l] = cconj(csub(P, wq));
      }
      float2 s1 = c2(0.f, 0.f), s2 = c2(0.f, 0.f);
#pragma unroll
      for (int l = 0; l < D2; ++l) { s1 = cadd(s1, cmul(gca[k][l], Xa[l])); s2 = cadd(s2, cmul(gcb[k][l], Xb[l])); }
      const float2 S = cscale(cadd(s1, cconj(s2)), 1.0f / (2 * D2));
      const float2 E = cscale(csub(gy[k], S), tau);
      const float2 Ec = cconj(E);
      const float inv_n = 1.0f / (2.0f * N);
#pragma unroll
      for (int l = 0; l < D2; ++l) {
        const int p = k2 + l * M;
        const int qq = (mode == 1) ? ((N2 - p) & (N2 - 1)) : (N2 - 1 - p);
        const float2 Va = cconjmul(gca[k][l], E);
        const float2 vbc = cconj(cconjmul(gcb[k][l], Ec));
        const float2 E_ = cscale(cadd(Va, vbc), inv_n);
        const float2 O_ = cscale(cmulc(csub(Va, vbc), gw[l]), inv_n);
        lds[lpr(sa * LDA + p)] = cadd(E_, cmuli(O_));
        if (write_b) lds[lpr(sb * LDA + qq)] = cconj(csub(E_, cmuli(O_)));
      }
    }
    __syncthreads();
    lds_fft<N2, RA, T, true, false, LDA>(lds, t2, tid);
#pragma unroll
    for (int k = 0; k < EA; ++k) {
      const unsigned i = tid + k * T;
      if (FA || i < RA * N2) s.Y[row_of(i / N2) * N2 + (i % N2)] = lds[lpr((i / N2) * LDA + (i % N2))];
    }
  }
}

// Column pass on CBB adjacent columns starting at j2_0 (interleaved LDS
// layout: element (column c, index i) at i*CBB + c).  MODE: B_FWD_REAL (load
// the real signal `in`), B_FWD_UP (load P^T y), B_ISTA (inverse, add the step
// to the iterate, threshold, forward; the last iteration skips the forward).
template <int N1, int N2, int CBB, int MODE, int H, int T>
__device__ __forceinline__ void batch_cols(const BatchSig& s, const float* in, int j2_0, bool last,
                                           float thr, float2* __restrict__ lds,
                                           const float2* __restrict__ t1, unsigned tid) {
  constexpr int N = N1 * N2;
  constexpr int NE = N1 * CBB;
  constexpr int EB = (NE + T - 1) / T;
  constexpr bool FB = NE % T == 0;
  constexpr int LOB = (ilog2c(N) + 1) / 2;
  static_assert(NE <= kBLds, "column step exceeds the LDS buffer");
  auto gidx = [&](unsigned e) -> unsigned { return (e / CBB) * N2 + j2_0 + (e % CBB); };
  auto twN = [&](unsigned e) -> float2 {
    const unsigned ex = ((j2_0 + (e % CBB)) * (e / CBB)) & (N - 1);
    return cmul(s.twlo[ex & ((1u << LOB) - 1)], s.twhi[ex >> LOB]);
  };
  if constexpr (MODE == B_ISTA) {
    float2 cv[EB];
#pragma unroll
    for (int k = 0; k < EB; ++k) {
      const unsigned e = tid + k * T;
      if (FB || e < NE) cv[k] = s.Y[gidx(e)];
    }
#pragma unroll
    for (int k = 0; k < EB; ++k) {
      const unsigned e = tid + k * T;
      if (FB || e < NE) lds[lp(e)] = cmulc(cv[k], twN(e));
    }
    __syncthreads();
    lds_fft<N1, CBB, T, true, true, N1>(lds, t1, tid);
    float2* xs = reinterpret_cast<float2*>(s.x);
    float2 sv[EB];
#pragma unroll
    for (int k = 0; k < EB; ++k) {
      const unsigned e = tid + k * T;
      if (FB || e < NE) sv[k] = xs[gidx(e)];
    }
#pragma unroll
    for (int k = 0; k < EB; ++k) {
      const unsigned e = tid + k * T;
      if (FB || e < NE) {
        const float2 v = cadd(sv[k], lds[lp(e)]);
        const float2 xv = c2(soft(v.x, thr), soft(v.y, thr));
        xs[gidx(e)] = xv;
        lds[lp(e)] = xv;
      }
    }
    if (last) return;
  } else {
    // B_FWD_REAL: the real signal; B_FWD_UP: P^T y, whose real sample 2j is
    // y[2j/d] when d divides 2j (H = d/2) and zero otherwise
    float2 v[EB];
#pragma unroll
    for (int k = 0; k < EB; ++k) {
      const unsigned e = tid + k * T;
      if (FB || e < NE) {
        const unsigned j = gidx(e);
        if constexpr (MODE == B_FWD_REAL) v[k] = reinterpret_cast<const float2*>(in)[j];
        else v[k] = c2((j % H) == 0 ? in[j / H] : 0.0f, 0.0f);
      }
    }
#pragma unroll
    for (int k = 0; k < EB; ++k) {
      const unsigned e = tid + k * T;
      if (FB || e < NE) lds[lp(e)] = v[k];
    }
  }
  __syncthreads();
  lds_fft<N1, CBB, T, false, true, N1>(lds, t1, tid);
#pragma unroll
  for (int k = 0; k < EB; ++k) {
    const unsigned e = tid + k * T;
    if (FB || e < NE) s.Y[gidx(e)] = cmul(lds[lp(e)], twN(e));
  }
}

// One signal, all iterations, by one workgroup.
template <int LOGN, int D2, int T>
__device__ __noinline__ void batch_solve_one(const BatchSig& s, int iters, float2* __restrict__ lds,
                                             float2* __restrict__ t1, float2* __restrict__ t2,
                                             unsigned tid) {
  constexpr int N1 = (LOGN % 2) ? (1 << ((LOGN - 1) / 2)) : (1 << (LOGN / 2 - 1));
  constexpr int N2 = (1 << LOGN) / N1;
  constexpr int N = N1 * N2;
  constexpr int AI0 = 1 << ilog2c(kBLds / (2 * (N2 + kPadA)));   // power of two that fits
  constexpr int AI = AI0 < N1 / 2 ? AI0 : N1 / 2;            // row pairs per step
  constexpr int CB0 = kBPoints / N1;
  constexpr int CBB = CB0 < N2 ? CB0 : N2;                   // columns per step
  static_assert(AI >= 1 && (N1 / 2) % AI == 0 && N2 % CBB == 0, "step split");
  static_assert(N2 / D2 >= 2, "decimation too large for this length");
  const float tau = *s.tau;
  const float thr = tau * *s.lam;

  for (unsigned i = tid; i < N1; i += T) t1[i] = s.tw1[i];
  for (unsigned i = tid; i < N2; i += T) t2[i] = s.tw2[i];
  __syncthreads();
  // c_hat table
  for (int j = 0; j < N2; j += CBB) {
    batch_cols<N1, N2, CBB, B_FWD_REAL, 1, T>(s, s.c, j, false, 0.f, lds, t1, tid);
    __syncthreads();
  }
  for (int w = 0; w < N1 / 2; w += AI) {
    batch_rows<N1, N2, D2, AI, A_SPEC, T>(s, s.chat, w, false, 0.f, lds, t2, tid);
    __syncthreads();
  }
  // y_hat table (DFT_n of P^T y)
  for (int j = 0; j < N2; j += CBB) {
    batch_cols<N1, N2, CBB, B_FWD_UP, D2, T>(s, s.y, j, false, 0.f, lds, t1, tid);
    __syncthreads();
  }
  for (int w = 0; w < N1 / 2; w += AI) {
    batch_rows<N1, N2, D2, AI, A_SPEC, T>(s, s.yhat, w, false, 0.f, lds, t2, tid);
    __syncthreads();
  }
  // x(0) = 0
  for (unsigned i = tid; i < 2 * N; i += T) s.x[i] = 0.0f;
  __syncthreads();
  for (int t = 1; t <= iters; ++t) {
    for (int w = 0; w < N1 / 2; w += AI) {
      batch_rows<N1, N2, D2, AI, A_ISTA, T>(s, nullptr, w, t == 1, tau, lds, t2, tid);
      __syncthreads();
    }
    for (int j = 0; j < N2; j += CBB) {
      batch_cols<N1, N2, CBB, B_ISTA, 1, T>(s, nullptr, j, t == iters, thr, lds, t1, tid);
      __syncthreads();
    }
  }
}

// The batched launch: workgroups pull signal indices from `queue` (zero at
// launch) until the batch is exhausted.
template <int D2>
__global__ __launch_bounds__(kBThreads) void k_batch_ista(const BatchSig* __restrict__ sigs, int count,
                                                         unsigned* queue, int iters) {
  constexpr int T = kBThreads;
  __shared__ float2 lds[lds_padded(kBLds)];
  __shared__ float2 t1[kBMaxN1];
  __shared__ float2 t2[kBMaxN2];
  __shared__ int next;
  const unsigned tid = threadIdx.x;
  for (;;) {
    if (tid == 0) next = int(atomicAdd(queue, 1u));
    __syncthreads();
    const int i = next;
    __syncthreads();
    if (i >= count) break;
    const BatchSig s = sigs[i];
    switch (s.logN) {
#define CS_B(L)                                                      \
  case L:                                                            \
    if constexpr ((1 << L) / ((L % 2) ? (1 << ((L - 1) / 2)) : (1 << (L / 2 - 1))) / D2 >= 2) \
      batch_solve_one<L, D2, T>(s, iters, lds, t1, t2, tid);         \
    break;
      CS_B(9) CS_B(10) CS_B(11) CS_B(12) CS_B(13) CS_B(14) CS_B(15) CS_B(16) CS_B(17)
#undef CS_B
      default: break;
    }
    __syncthreads();
  }
}

}  // namespace cs
