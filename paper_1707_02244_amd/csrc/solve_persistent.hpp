// Persistent single-launch ISTA / ADMM solver (one cooperative launch per
// solve).
//
// Same arithmetic as the two-pass kernels in kernels.hpp: the four-step
// N = N1 * N2 factorisation, the packed real split, the alias-class update and
// the fused time-domain epilogue.  One launch runs all iterations, with a grid
// barrier between the row pass and the column pass.  Each workgroup owns fixed
// work for the whole solve:
//   - AI row pairs {w, N1 - w}, w = g + i*G (the row pass); the c_hat and
//     y_hat entries of its alias classes are loaded into registers once per
//     solve and stay there;
//   - one block of CB adjacent columns (the column pass); it keeps the
//     time-domain state of those columns (ISTA: the iterate x; ADMM: the
//     scaled dual u) in registers.
// The state never leaves the CU between iterations: HBM sees only the
// spectrum buffer Y (read and written by both passes, 16n bytes per
// iteration).  All twiddle tables (FFT stages, four-step, real split) are
// loaded into LDS once per launch.
//
// Y interleaves each mirror row pair: element (k1, j2) of the four-step
// intermediate lives at Y[(w * N2 + j2) * 2 + s], where pair w holds rows w
// (s = 0) and N1 - w (s = 1), and pair 0 holds rows 0 and N1/2.  A row-pass
// workgroup then reads and writes one contiguous block of 2 N2 values per
// pair, and a column-pass workgroup (8 adjacent columns) moves 128-byte runs
// (8 columns x 2 rows) instead of 64-byte ones.
//
// Grid size G = N2 / CB; the split is chosen so that N1/2 = AI * G with AI = 1
// or 2.  The launch is cooperative (hipLaunchCooperativeKernel), so all G
// workgroups are resident and the barrier's wait always ends; the wait is also
// bounded (kSpinLimit polls): hitting the bound sets an error flag, and every
// later wait returns at once, so a faulty launch still drains.
#pragma once
#include <stdint.h>

#include "kernels.hpp"

namespace cs {

constexpr int kPThreads = 512;
constexpr unsigned kSpinLimit = 1u << 20;   // polls (~40 ms); a real wait is ~100 us

struct SolveArgs {
  float2* Y;               // [N1][N2] spectrum exchange buffer
  const float2* chat;      // c_hat table ([k1*N2 + k2], Nyquist at [N])
  const float2* yhat;      // DFT_n(P^T y) table, same layout
  const float2* tw1;       // W_{N1}^e
  const float2* tw2;       // W_{N2}^e
  const float2* twlo;      // W_N^e, e < 2^lo_bits
  const float2* twhi;      // W_N^{e * 2^lo_bits}
  const float2* twk1;      // W_n^{k1}
  const float2* twp;       // W_{2 N2}^p
  int lo_bits;
  float* x;                // ISTA: output x(T).  ADMM: output x(T)
  float* z;                // ADMM: in (warm) / out z(T)
  float* u;                // ADMM: in (warm) / out u(T)
  unsigned* bar;           // grid barrier counters (kBarWords words), zero at launch
  int* err;                // set to 1 if a barrier wait hit its bound
  int iters;
  int warm;
  float tau;               // ISTA step
  float thr;               // ISTA: tau*lam; ADMM: lam/rho
  float inv_n, inv_d;
  float rho, inv_rho, d_rho;
};

// The spectrum buffer Y is the only data workgroups exchange.  It is read
// and written with relaxed agent-scope atomic accesses: on gfx950 these are
// plain vector loads/stores carrying the device-coherence bit, so a value
// stored by one XCD is what another XCD's load returns, without writing back
// or invalidating any L2 (the read-only c_hat / y_hat tables keep their L2
// residency across iterations).
__device__ __forceinline__ float2 ld_coh(const float2* p) {
  const uint64_t v = __hip_atomic_load(reinterpret_cast<const uint64_t*>(p), __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
  return __builtin_bit_cast(float2, v);
}
__device__ __forceinline__ void st_coh(float2* p, float2 v) {
  __hip_atomic_store(reinterpret_cast<uint64_t*>(p), __builtin_bit_cast(uint64_t, v), __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
}

// Grid-wide barrier.  Arrivals are spread over NC counters, each on its own
// 128-byte line (workgroup g adds to counter g mod NC): a single counter
// serialises all G atomic adds on one line, several microseconds per barrier
// at G = 256.  Each wave first waits until its own coherent stores have
// completed, the workgroup synchronises, lane 0 of wave 0 arrives, and wave 0
// polls all counters at once (lane c reads counter c) until every one has
// reached its target; a workgroup barrier releases the other waves.  The wait
// is bounded; hitting the bound sets the error flag, and a set flag ends every
// later wait at once.
#ifndef CS_BAR_COUNTERS
#define CS_BAR_COUNTERS 256
#endif
#ifndef CS_BAR_SLEEP
#define CS_BAR_SLEEP 2
#endif
constexpr int kBarCounters = CS_BAR_COUNTERS;         // arrival counters (max; one wave polls them)
constexpr int kBarStride = 32;                        // unsigned per counter: 128 bytes
constexpr int kBarErr = kBarCounters * kBarStride;    // error flag, its own line
constexpr int kBarWords = kBarErr + kBarStride;       // size of the barrier area

template <int NC>
__device__ __forceinline__ void grid_barrier(unsigned* bar, unsigned target, int* err) {
  static_assert(NC >= 1 && NC <= kBarCounters, "");
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x < 64) {
    const unsigned lane = threadIdx.x;
    if (lane == 0)
      __hip_atomic_fetch_add(bar + (blockIdx.x % NC) * kBarStride, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    unsigned spins = 0;
    while (true) {
      bool ok = true;
#pragma unroll
      for (int c0 = 0; c0 < NC; c0 += 64) {
        const bool r = (c0 + lane >= (unsigned)NC) ||
                       __hip_atomic_load(bar + (c0 + lane) * kBarStride, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= target;
        ok &= r;
      }
      if (__all(ok)) break;
      __builtin_amdgcn_s_sleep(CS_BAR_SLEEP);
      if (++spins > kSpinLimit) {
        if (lane == 0) __hip_atomic_fetch_or(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
      if ((spins & 255) == 0 && __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
    }
  }
  __syncthreads();
}

template <int N1, int N2, int D2, int AI, int ALG>  // ALG 0: ISTA, 1: ADMM
__global__ __launch_bounds__(kPThreads) void k_solve(SolveArgs a) {
  constexpr int T = kPThreads;
  constexpr int CB = kColsPerBlock;
  constexpr int N = N1 * N2;
  constexpr int G = N2 / CB;
  static_assert(N1 / 2 == AI * G, "split must give AI row pairs per workgroup");
  constexpr int LDA = N2 + kPadA;
  constexpr int RA = 2 * AI;                 // rows held in the row pass
  constexpr int NA = RA * LDA;
  constexpr int NEB = N1 * CB;
  constexpr int NL = lds_rows(NA) > NEB ? lds_rows(NA) : NEB;
  constexpr int EA = (RA * N2 + T - 1) / T;  // row-pass elements per thread
  constexpr bool FA = (RA * N2) % T == 0;
  constexpr int EB = (NEB + T - 1) / T;      // column-pass elements per thread
  constexpr bool FB = NEB % T == 0;
  constexpr int M = N2 / D2;                 // alias classes per row (m / N1)
  constexpr int GPT = (AI * M + 1 + T - 1) / T;
  __shared__ float2 lds[lds_padded(NL)];
  __shared__ float2 t1[N1];
  __shared__ float2 t2[N2];
  __shared__ float2 tp[N2];                  // W_{2 N2}^p (real-split twiddle, row part)
  constexpr int LOB = (ilog2c(N) + 1) / 2;   // two-level four-step twiddle W_N^e
  __shared__ float2 tlo[1 << LOB];           // W_N^e, e < 2^LOB
  __shared__ float2 thi[N >> LOB];           // W_N^{e * 2^LOB}
  unsigned tid = threadIdx.x;
  const int g = blockIdx.x;
  const unsigned j2_0 = g * CB;

  // ---- one-time set-up ---------------------------------------------------
  for (int i = tid; i < N1; i += T) t1[i] = a.tw1[i];
  for (int i = tid; i < N2; i += T) t2[i] = a.tw2[i];

  for (int i = tid; i < N2; i += T) tp[i] = a.twp[i];
  for (int i = tid; i < (1 << LOB); i += T) tlo[i] = a.twlo[i];
  for (int i = tid; i < (N >> LOB); i += T) thi[i] = a.twhi[i];
  // W_N^{(j2 * k1) mod N} for column-pass element e
  auto twb = [&](unsigned e) -> float2 {
    const unsigned ex = ((j2_0 + (e % CB)) * (e / CB)) & (N - 1);
    return cmul(tlo[ex & ((1u << LOB) - 1)], thi[ex >> LOB]);
  };
  // row pass: this thread's alias classes, q = tid + k*T over the row pairs
  // w_i = g + i*G (pair 0 of workgroup 0 holds rows 0 and N1/2 and has one
  // extra class)
  const int ng0 = (g == 0) ? (M + 1) : M;
  const int ncls = ng0 + (AI - 1) * M;
  struct Cls { int sa, sb, rowa, rowb, k2, mode; };
  auto decode = [&](unsigned q) -> Cls {
    const int pi = (q < (unsigned)ng0) ? 0 : 1 + (q - ng0) / M;
    const int lc = (q < (unsigned)ng0) ? q : (q - ng0) % M;
    const int w = g + pi * G;
    Cls c;
    if (w) { c.sa = 2 * pi; c.sb = 2 * pi + 1; c.rowa = w; c.rowb = N1 - w; c.k2 = lc; c.mode = 0; }
    else if (lc <= (M >> 1)) { c.sa = c.sb = 2 * pi; c.rowa = c.rowb = 0; c.k2 = lc; c.mode = 1; }
    else { c.sa = c.sb = 2 * pi + 1; c.rowa = c.rowb = N1 >> 1; c.k2 = lc - (M >> 1) - 1; c.mode = 2; }
    return c;
  };

  // column pass: this thread's elements e = tid + k*T, k1 = e / CB,
  // column j2 = j2_0 + e % CB, and their time-domain state
  float2 st[EB];
#pragma unroll
  for (int k = 0; k < EB; ++k) st[k] = c2(0.f, 0.f);

  unsigned nbar = 0;
  constexpr int NC = G < kBarCounters ? G : kBarCounters;   // barrier counters (G is a power of two)
  constexpr unsigned PER_C = G / NC;                          // arrivals per counter per barrier
  float2* Yg = a.Y;
  // element offsets fit in 32 bits (N <= 2^21 here); a uniform base plus a
  // 32-bit offset lets the compiler use scalar-base addressing
  static_assert(T % CB == 0, "");
  auto col_index = [&](unsigned e) -> unsigned { return (e / CB) * N2 + j2_0 + (e % CB); };
  // column-pass access to Y: slot e of the workgroup's block in Y order
  // (pair w = e / (2 CB), column c = (e / 2) % CB, side s = e % 2) -> its
  // Y offset and its LDS element (row k1, column c) in the interleaved
  // column layout k1 * CB + c
  auto ycol_off = [&](unsigned e) -> unsigned {
    return (e / (2 * CB)) * (2 * N2) + (j2_0 + (e / 2) % CB) * 2 + (e & 1);
  };
  auto ycol_lds = [&](unsigned e) -> unsigned {
    const unsigned w = e / (2 * CB), c = (e / 2) % CB;
    const unsigned k1 = (e & 1) ? (w ? N1 - w : (N1 >> 1)) : w;
    return k1 * CB + c;
  };

  // forward column transform of lds (time domain) and store to Y
  auto col_forward_store = [&]() {
    lds_fft<N1, CB, T, false, true, N1>(lds, t1, tid);
#pragma unroll
    for (int k = 0; k < EB; ++k) {
      const unsigned e = tid + k * T;
      if (FB || e < NEB) {
        const unsigned li = ycol_lds(e);
        st_coh(&Yg[ycol_off(e)], cmul(lds[lp(li)], twb(li)));
      }
    }
  };

  if (ALG == 1 && a.warm) {
    // ADMM warm start: state u and spectrum of z - u
    const float2* z2 = reinterpret_cast<const float2*>(a.z);
    const float2* u2 = reinterpret_cast<const float2*>(a.u);
#pragma unroll
    for (int k = 0; k < EB; ++k) {
      const unsigned e = tid + k * T;
      if (FB || e < NEB) {
        const unsigned j = col_index(e);
        st[k] = u2[j];
        lds[lp(e)] = csub(z2[j], st[k]);
      }
    }
    __syncthreads();
    col_forward_store();
    grid_barrier<NC>(a.bar, (++nbar) * PER_C, a.err);
  }
  __syncthreads();

  // class operands (c_hat, y_hat at this thread's alias classes) are
  // constant over the solve: load them once
  float2 gca[GPT][D2], gcb[GPT][D2], gy[GPT];
  {
#pragma unroll
    for (int k = 0; k < GPT; ++k) {
      const unsigned q = tid + k * T;
      if (q < (unsigned)ncls) {
        const Cls c = decode(q);
#pragma unroll
        for (int l = 0; l < D2; ++l) {
          const int p = c.k2 + l * M;
          const int qq = (c.mode == 1) ? ((N2 - p) & (N2 - 1)) : (N2 - 1 - p);
          gca[k][l] = a.chat[(unsigned)c.rowa * N2 + p];
          gcb[k][l] = (c.mode == 1 && p == 0) ? a.chat[N] : a.chat[(unsigned)c.rowb * N2 + qq];
        }
        gy[k] = a.yhat[(unsigned)c.rowa * N2 + c.k2];
      }
    }
  }
  for (int t = 1; t <= a.iters; ++t) {
    // keep per-thread index arithmetic inside the iteration: hoisting it out
    // of the loop keeps dozens of addresses live and forces spills
    asm volatile("" : "+v"(tid));
    // ---- row pass: forward rows, alias-class update, inverse rows ----------
    // Issue every row load before the first LDS store.
    {
      float2 rv[EA];
      const bool zero_in = (t == 1) && !(ALG == 1 && a.warm);
#pragma unroll
      for (int k = 0; k < EA; ++k) {
        const unsigned i = tid + k * T;
        if (FA || i < RA * N2) {
          // pair i / (2 N2) of this workgroup, one contiguous block
          const unsigned w = g + (i / (2 * N2)) * G;
          rv[k] = zero_in ? c2(0.f, 0.f) : ld_coh(&Yg[w * (2 * N2) + i % (2 * N2)]);
        }
      }
#pragma unroll
      for (int k = 0; k < EA; ++k) {
        const unsigned i = tid + k * T;
        // slot 2 * pair + side, position j2
        if (FA || i < RA * N2) lds[lpr((2 * (i / (2 * N2)) + (i & 1)) * LDA + (i % (2 * N2)) / 2)] = rv[k];
      }
    }
    __syncthreads();
    lds_fft<N2, RA, T, false, false, LDA>(lds, t2, tid);
#pragma unroll
    for (int k = 0; k < GPT; ++k) {
      const unsigned q = tid + k * T;
      if (q >= (unsigned)ncls) continue;
      const Cls c = decode(q);
      const int sa = c.sa, sb = c.sb, k2 = c.k2, mode = c.mode;
      const bool write_b = !(mode == 1 && (k2 == 0 || k2 == (M >> 1)));
      const float2 wk1 = a.twk1[c.rowa];
      float2 Xa[D2], Xb[D2], gw[D2];
#pragma unroll
      for (int l = 0; l < D2; ++l) {
        const int p = k2 + l * M;
        const int qq = (mode == 1) ? ((N2 - p) & (N2 - 1)) : (N2 - 1 - p);
        gw[l] = cmul(wk1, tp[p]);
        const float2 za = lds[lpr(sa * LDA + p)];
        const float2 zbc = cconj(lds[lpr(sb * LDA + qq)]);
        const float2 P = cscale(cadd(za, zbc), 0.5f);
        const float2 Q = cscale(cmulmi(csub(za, zbc)), 0.5f);
        const float2 wq = cmul(gw[l], Q);
        Xa[l] = cadd(P, wq);
        Xb[l] = cconj(csub(P, wq));
      }
      float2 Va[D2], Vb[D2];
      if constexpr (ALG == 0) {
        float2 s1 = c2(0.f, 0.f), s2 = c2(0.f, 0.f);
#pragma unroll
        for (int l = 0; l < D2; ++l) { s1 = cadd(s1, cmul(gca[k][l], Xa[l])); s2 = cadd(s2, cmul(gcb[k][l], Xb[l])); }
        const float2 S = cscale(cadd(s1, cconj(s2)), a.inv_d);
        const float2 E = cscale(csub(gy[k], S), a.tau);
        const float2 Ec = cconj(E);
#pragma unroll
        for (int l = 0; l < D2; ++l) {
          Va[l] = cconjmul(gca[k][l], E);
          Vb[l] = cconjmul(gcb[k][l], Ec);
        }
      } else {
        // residual form of the Woodbury x-update: X' = X + conj(c) E
        float2 r1 = c2(0.f, 0.f), r2 = c2(0.f, 0.f);
        float den = a.d_rho;
#pragma unroll
        for (int l = 0; l < D2; ++l) {
          r1 = cadd(r1, cmul(gca[k][l], Xa[l]));
          r2 = cadd(r2, cmul(gcb[k][l], Xb[l]));
          den += cabs2(gca[k][l]) + cabs2(gcb[k][l]);
        }
        const float2 S = cscale(cadd(r1, cconj(r2)), a.inv_d);
        const float2 E = cscale(csub(gy[k], S), 1.0f / (den * a.inv_d));
        const float2 Ec = cconj(E);
#pragma unroll
        for (int l = 0; l < D2; ++l) {
          Va[l] = cadd(Xa[l], cconjmul(gca[k][l], E));
          Vb[l] = cadd(Xb[l], cconjmul(gcb[k][l], Ec));
        }
      }
#pragma unroll
      for (int l = 0; l < D2; ++l) {
        const int p = k2 + l * M;
        const int qq = (mode == 1) ? ((N2 - p) & (N2 - 1)) : (N2 - 1 - p);
        const float2 vbc = cconj(Vb[l]);
        const float2 E_ = cscale(cadd(Va[l], vbc), a.inv_n);
        const float2 O_ = cscale(cmulc(csub(Va[l], vbc), gw[l]), a.inv_n);
        lds[lpr(sa * LDA + p)] = cadd(E_, cmuli(O_));
        if (write_b) lds[lpr(sb * LDA + qq)] = cconj(csub(E_, cmuli(O_)));
      }
    }
    __syncthreads();
    lds_fft<N2, RA, T, true, false, LDA>(lds, t2, tid);
#pragma unroll
    for (int k = 0; k < EA; ++k) {
      const unsigned i = tid + k * T;
      if (FA || i < RA * N2) {
        const unsigned w = g + (i / (2 * N2)) * G;
        st_coh(&Yg[w * (2 * N2) + i % (2 * N2)],
               lds[lpr((2 * (i / (2 * N2)) + (i & 1)) * LDA + (i % (2 * N2)) / 2)]);
      }
    }
    grid_barrier<NC>(a.bar, (++nbar) * PER_C, a.err);

    // ---- column pass: inverse columns, epilogue, forward columns -----------
    {
      float2 cv[EB];
#pragma unroll
      for (int k = 0; k < EB; ++k) {
        const unsigned e = tid + k * T;
        if (FB || e < NEB) cv[k] = ld_coh(&Yg[ycol_off(e)]);
      }
#pragma unroll
      for (int k = 0; k < EB; ++k) {
        const unsigned e = tid + k * T;
        if (FB || e < NEB) {
          const unsigned li = ycol_lds(e);
          lds[lp(li)] = cmulc(cv[k], twb(li));
        }
      }
    }
    __syncthreads();
    lds_fft<N1, CB, T, true, true, N1>(lds, t1, tid);
    const bool last = (t == a.iters);
    const float thr = a.thr;
#pragma unroll
    for (int k = 0; k < EB; ++k) {
      const unsigned e = tid + k * T;
      if (FB || e < NEB) {
        if constexpr (ALG == 0) {
          const float2 v = cadd(st[k], lds[lp(e)]);
          const float2 xv = c2(soft(v.x, thr), soft(v.y, thr));
          st[k] = xv;
          lds[lp(e)] = xv;
        } else {
          const float2 xv = lds[lp(e)];
          const float2 xu = cadd(xv, st[k]);
          const float2 zv = c2(soft(xu.x, thr), soft(xu.y, thr));
          const float2 u1 = csub(xu, zv);
          st[k] = u1;
          if (last) {
            const unsigned j = col_index(e);
            reinterpret_cast<float2*>(a.x)[j] = xv;
            reinterpret_cast<float2*>(a.z)[j] = zv;
          } else {
            lds[lp(e)] = csub(zv, u1);
          }
        }
      }
    }
    if (!last) {
      __syncthreads();
      col_forward_store();
      grid_barrier<NC>(a.bar, (++nbar) * PER_C, a.err);
    }
  }

  // ---- outputs -------------------------------------------------------------
  float2* out = reinterpret_cast<float2*>(ALG == 0 ? a.x : a.u);
  if (ALG == 0 || a.iters > 0) {
#pragma unroll
    for (int k = 0; k < EB; ++k) {
      const unsigned e = tid + k * T;
      if (FB || e < NEB) out[col_index(e)] = st[k];
    }
  }
}

}  // namespace cs
