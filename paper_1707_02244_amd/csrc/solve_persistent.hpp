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
// bounded in time (the device wall clock, max_ticks per wait): hitting the
// bound sets an error flag, and every later wait returns at once, so a faulty
// launch still drains within about one bound.
#pragma once
#include <stdint.h>

#include <type_traits>

#include "kernels.hpp"

namespace cs {

constexpr int kPThreads = 512;

// Register-stage path (first and last radix-8 stage of every transform in
// registers) for the larger sizes; CS_REG_MIN_N1 is the smallest N1 that
// takes it (below it, too few threads would hold butterflies).
#ifndef CS_REG_STAGES
#define CS_REG_STAGES 1
#endif
#ifndef CS_REG_MIN_N1
#define CS_REG_MIN_N1 512
#endif

// Pins a value to registers (an empty asm that claims to modify it), so a
// select between two such values stays a select of registers.
__device__ __forceinline__ void opaque(float2& v) { asm("" : "+v"(v.x), "+v"(v.y)); }

// Compile-time loop: f(std::integral_constant<int, I>) for I in [B, E).
template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

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
  uint64_t max_ticks;      // bound of one barrier wait in wall-clock ticks
  int iters;
  int warm;
  float tau;               // ISTA step
  float thr;               // ISTA: tau*lam; ADMM: lam/rho
  float inv_n, inv_d;
  float rho, inv_rho, d_rho;
  double* res;             // objective trace (traced instances): per iteration t
  double* l1;              //   and workgroup g, res[(t-1) G + g] = sum over g's
                           //   m-point bins of |Y_hat - S|^2 for x(t) and
                           //   l1[(t-1) G + g] = sum of |x(t)| over g's columns
};

// 16-byte forms of ld_coh / st_coh (two adjacent float2) for the register-
// stage path: raw buffer accesses with the same device-coherence cache bit
// (sc1) that the relaxed agent-scope atomics above carry.  The buffer
// resource covers exactly the spectrum buffer, so an offset outside it reads
// zeros and drops the store instead of touching other memory.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t y_rsrc(float2* Y, unsigned n_elems) {
  return __builtin_amdgcn_make_buffer_rsrc(Y, 0, (int)(n_elems * 8u), kBufWord3);
}
__device__ __forceinline__ void ld_coh_pair(__amdgpu_buffer_rsrc_t rs, unsigned elem, float2& lo, float2& hi) {
  const cs_u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(rs, elem * 8u, 0, kCohAux);
  lo = c2(__uint_as_float(v.x), __uint_as_float(v.y));
  hi = c2(__uint_as_float(v.z), __uint_as_float(v.w));
}
__device__ __forceinline__ void st_coh_pair(__amdgpu_buffer_rsrc_t rs, unsigned elem, float2 lo, float2 hi) {
  // the values are pinned to registers first: otherwise the compiler may
  // read the caller's array element and its neighbour as one 16-byte load,
  // and an array read that way cannot stay in registers
  asm("" : "+v"(lo.x), "+v"(lo.y), "+v"(hi.x), "+v"(hi.y));
  const cs_u32x4 v = {__float_as_uint(lo.x), __float_as_uint(lo.y), __float_as_uint(hi.x),
                      __float_as_uint(hi.y)};
  __builtin_amdgcn_raw_buffer_store_b128(v, rs, elem * 8u, 0, kCohAux);
}

// One alias class of the row pass on registers (the same arithmetic as the
// LDS form in k_solve).  The class's row-a values at p_l = k2 + l*M sit at
// indices RHO + l*(8/D2) of A; their mirrors (row b at N2-1-p_l, or at
// (N2-p_l) mod N2 in row 0) at indices 7-RHO-l*(8/D2) of Bv (MK = 0) or
// (8-RHO-l*(8/D2)) mod 8 (MK = 1).  A and Bv may be the same array: every
// input is read before any output is written.  WB = false for the classes
// that are their own mirror (row 0, k2 = 0 and M/2).  ALG 2 only adds the
// class's squared residual to racc (the final iterate's trace entry); with
// TR, ALG 0 and 1 add it too (ISTA: of the input iterate; ADMM: of the
// updated x).  A class and its mirror bin count twice, a self-mirror class
// once (Parseval over the m-point spectrum).
template <int D2, int M, int RHO, int MK, bool WB, int ALG, bool TR, typename Args>
__device__ __forceinline__ void class_step(float2 (&A)[8], float2 (&Bv)[8], const float2 (&gca)[D2],
                                           const float2 (&gcb)[D2], float2 gy, unsigned k2, float2 wk1,
                                           const float2* __restrict__ tp, const Args& a, float& racc) {
  constexpr int RM = 8 / D2;
  constexpr float RW = WB ? 2.0f : 1.0f;
  float2 Xa[D2], Xb[D2], gw[D2];
#pragma unroll
  for (int l = 0; l < D2; ++l) {
    const int ia = RHO + l * RM;
    const int ib = MK == 0 ? 7 - RHO - l * RM : (8 - RHO - l * RM) & 7;
    gw[l] = cmul(wk1, tp[k2 + l * M]);
    const float2 za = A[ia];
    const float2 zbc = cconj(Bv[ib]);
    const float2 P = cscale(cadd(za, zbc), 0.5f);
    const float2 Q = cscale(cmulmi(csub(za, zbc)), 0.5f);
    const float2 wq = cmul(gw[l], Q);
    Xa[l] = cadd(P, wq);
    Xb[l] = cconj(csub(P, wq));
  }
  float2 Va[D2], Vb[D2];
  if constexpr (ALG == 2) {
    float2 s1 = c2(0.f, 0.f), s2 = c2(0.f, 0.f);
#pragma unroll
    for (int l = 0; l < D2; ++l) { s1 = cadd(s1, cmul(gca[l], Xa[l])); s2 = cadd(s2, cmul(gcb[l], Xb[l])); }
    racc += RW * cabs2(csub(gy, cscale(cadd(s1, cconj(s2)), a.inv_d)));
    return;
  } else if constexpr (ALG == 0) {
    float2 s1 = c2(0.f, 0.f), s2 = c2(0.f, 0.f);
#pragma unroll
    for (int l = 0; l < D2; ++l) { s1 = cadd(s1, cmul(gca[l], Xa[l])); s2 = cadd(s2, cmul(gcb[l], Xb[l])); }
    const float2 S = cscale(cadd(s1, cconj(s2)), a.inv_d);
    if constexpr (TR) racc += RW * cabs2(csub(gy, S));
    const float2 E = cscale(csub(gy, S), a.tau);
    const float2 Ec = cconj(E);
#pragma unroll
    for (int l = 0; l < D2; ++l) {
      Va[l] = cconjmul(gca[l], E);
      Vb[l] = cconjmul(gcb[l], Ec);
    }
  } else {
    float2 r1 = c2(0.f, 0.f), r2 = c2(0.f, 0.f);
    float den = a.d_rho;
#pragma unroll
    for (int l = 0; l < D2; ++l) {
      r1 = cadd(r1, cmul(gca[l], Xa[l]));
      r2 = cadd(r2, cmul(gcb[l], Xb[l]));
      den += cabs2(gca[l]) + cabs2(gcb[l]);
    }
    const float2 S = cscale(cadd(r1, cconj(r2)), a.inv_d);
    const float2 E = cscale(csub(gy, S), 1.0f / (den * a.inv_d));
    const float2 Ec = cconj(E);
#pragma unroll
    for (int l = 0; l < D2; ++l) {
      Va[l] = cadd(Xa[l], cconjmul(gca[l], E));
      Vb[l] = cadd(Xb[l], cconjmul(gcb[l], Ec));
    }
    if constexpr (TR) {
      float2 s1 = c2(0.f, 0.f), s2 = c2(0.f, 0.f);
#pragma unroll
      for (int l = 0; l < D2; ++l) { s1 = cadd(s1, cmul(gca[l], Va[l])); s2 = cadd(s2, cmul(gcb[l], Vb[l])); }
      racc += RW * cabs2(csub(gy, cscale(cadd(s1, cconj(s2)), a.inv_d)));
    }
  }
#pragma unroll
  for (int l = 0; l < D2; ++l) {
    const int ia = RHO + l * RM;
    const int ib = MK == 0 ? 7 - RHO - l * RM : (8 - RHO - l * RM) & 7;
    const float2 vbc = cconj(Vb[l]);
    const float2 E_ = cscale(cadd(Va[l], vbc), a.inv_n);
    const float2 O_ = cscale(cmulc(csub(Va[l], vbc), gw[l]), a.inv_n);
    A[ia] = cadd(E_, cmuli(O_));
    if constexpr (WB) Bv[ib] = cconj(csub(E_, cmuli(O_)));
  }
}

// Grid-wide barrier.  Arrivals are spread over NC counters, each on its own
// 128-byte line (workgroup g adds to counter g mod NC): a single counter
// serialises all G atomic adds on one line, several microseconds per barrier
// at G = 256.  Each wave first waits until its own coherent stores have
// completed, the workgroup synchronises, lane 0 of wave 0 arrives, and wave 0
// polls all counters at once (lane c reads counter c) until every one has
// reached its target; a workgroup barrier releases the other waves.  The wait
// is bounded in wall-clock time; hitting the bound sets the error flag, and
// every poll also reads the flag, so a set flag ends every later wait at once.
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
__device__ __forceinline__ void grid_barrier(unsigned* bar, unsigned target, int* err, uint64_t max_ticks) {
  static_assert(NC >= 1 && NC <= kBarCounters, "");
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x < 64) {
    const unsigned lane = threadIdx.x;
    if (lane == 0)
      __hip_atomic_fetch_add(bar + (blockIdx.x % NC) * kBarStride, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint64_t t0 = wall_clock64();
    while (true) {
      bool ok = true;
#pragma unroll
      for (int c0 = 0; c0 < NC; c0 += 64) {
        const bool r = (c0 + lane >= (unsigned)NC) ||
                       __hip_atomic_load(bar + (c0 + lane) * kBarStride, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= target;
        ok &= r;
      }
      if (__all(ok)) break;
      // a set flag (an earlier wait of this launch expired) ends the wait at once
      if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
      if (wall_clock64() - t0 > max_ticks) {
        if (lane == 0) __hip_atomic_fetch_or(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
      __builtin_amdgcn_s_sleep(CS_BAR_SLEEP);
    }
  }
  __syncthreads();
}

// ALG 0: ISTA, 1: ADMM.  TR: also write the objective trace's per-workgroup
// partial sums (a.res, a.l1); ISTA then takes one more forward column
// transform and a residual-only row pass after the last iteration, for the
// final iterate's residual.
template <int N1, int N2, int D2, int AI, int ALG, bool TR = false>
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
  constexpr bool REG = CS_REG_STAGES && N1 >= CS_REG_MIN_N1 && N1 >= 64 && N2 >= 64;
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
  if constexpr (REG) {
    // ---- register-stage path ------------------------------------------------
    // Row pass: thread (pair rpi, butterfly rt) loads the two rows of its
    // pair at positions rt + r*Q with 16-byte accesses and takes the first
    // forward stage in registers.  The last forward stage is taken in the
    // mirror mapping (row a at jA, row b at jB = its mirror butterfly), so
    // every alias class a thread updates has both of its sides in that
    // thread's registers; the first inverse stage follows in registers, and
    // the last inverse stage returns to the load mapping for the store.
    // Column pass: thread (column cc, pair cu) holds butterflies cjA and cjB
    // whose rows k1 and N1 - k1 share the 16-byte Y entries of a row pair;
    // the threshold epilogue runs on registers between the last inverse and
    // the first forward stage.
    constexpr unsigned Q = N2 / 8;            // row butterflies per row
    constexpr unsigned QC = N1 / 8;           // column butterflies per column
    constexpr int RM = 8 / D2;                // classes per row butterfly
    constexpr int NK = RM + 1;                // class slots (row 0 has one extra)
    static_assert(AI * Q <= (unsigned)T && CB * QC / 2 <= (unsigned)T, "too few threads");
    static_assert(M % Q == 0 && Q % 2 == 0 && QC % 2 == 0, "");
    const __amdgpu_buffer_rsrc_t rs = y_rsrc(a.Y, (unsigned)N);

    // row-pass roles: cat 0 = row pair {w, N1-w}; for pair 0 (rows 0 and
    // N1/2, each its own mirror): cat 2 = row 0 butterflies {0, Q/2}, cat 1
    // = row 0 butterflies {t, Q-t}, cat 3 = row N1/2 butterflies {u, Q-1-u}
    const bool ract = tid < AI * Q;
    unsigned rpi = tid / Q, rt = tid % Q;
    unsigned wp = g + rpi * G;
    int cat = -1;
    unsigned jA = 0, jB = 0, sA = 0, sB = 0, rowA = 0, rowB = 0;
    if (ract) {
      if (wp == 0) {
        if (rt < Q / 2) {
          cat = rt ? 1 : 2;
          jA = rt; jB = rt ? Q - rt : Q / 2; sA = sB = 2 * rpi; rowA = rowB = 0;
        } else {
          cat = 3;
          jA = rt - Q / 2; jB = Q - 1 - jA; sA = sB = 2 * rpi + 1; rowA = rowB = N1 / 2;
        }
      } else {
        cat = 0;
        jA = rt; jB = Q - 1 - rt; sA = 2 * rpi; sB = 2 * rpi + 1; rowA = wp; rowB = N1 - wp;
      }
    }
    // class operands of this thread's class slot k (c_hat at both sides,
    // y_hat); with CS_REG_HOIST they are loaded once per solve into
    // registers, otherwise before each use
    float2 wk1 = c2(1.f, 0.f);
    if (ract) wk1 = a.twk1[rowA];
    auto slot_k2 = [&](int k, bool& valid, int& mode) __attribute__((always_inline)) -> unsigned {
      unsigned k2 = 0;
      valid = false;
      mode = 0;
      if (cat == 0) {
        valid = k < RM; k2 = jA + k * Q;
      } else if (cat == 2) {
        valid = true; mode = 1;
        if (RM >= 2) k2 = (k <= RM / 2) ? k * Q : Q / 2 + (k - RM / 2 - 1) * Q;
        else k2 = (k == 0) ? 0 : Q / 2;
      } else if (cat > 0) {
        valid = k < RM; mode = (cat == 1) ? 1 : 2;
        if (RM >= 2) k2 = (k < RM / 2) ? jA + k * Q : jB + (k - RM / 2) * Q;
        else k2 = jA;
      }
      return valid ? k2 : 0;
    };
    auto load_ops = [&](int k, float2 (&gca)[D2], float2 (&gcb)[D2], float2& gy, unsigned& k2) __attribute__((always_inline)) {
      bool valid;
      int mode;
      k2 = slot_k2(k, valid, mode);
      gy = c2(0.f, 0.f);
#pragma unroll
      for (int l = 0; l < D2; ++l) { gca[l] = c2(0.f, 0.f); gcb[l] = c2(0.f, 0.f); }
      if (valid) {
#pragma unroll
        for (int l = 0; l < D2; ++l) {
          const unsigned pp = k2 + l * M;
          const unsigned qq = (mode == 1) ? ((N2 - pp) & (N2 - 1)) : (N2 - 1 - pp);
          gca[l] = a.chat[rowA * N2 + pp];
          gcb[l] = (mode == 1 && pp == 0) ? a.chat[N] : a.chat[rowB * N2 + qq];
        }
        gy = a.yhat[rowA * N2 + k2];
      }
    };
#ifndef CS_REG_HOIST
#define CS_REG_HOIST 1
#endif
    float2 rca[CS_REG_HOIST ? NK : 1][D2], rcb[CS_REG_HOIST ? NK : 1][D2], ryv[CS_REG_HOIST ? NK : 1];
    unsigned rk2[CS_REG_HOIST ? NK : 1];
    if constexpr (CS_REG_HOIST) {
      static_for<0, NK>([&](auto K) __attribute__((always_inline)) {
        constexpr int k = decltype(K)::value;
        load_ops(k, rca[k], rcb[k], ryv[k], rk2[k]);
      });
    }
    // class step for slot KS with mapping (RHO, MK, WB) on arrays (X, Y)
    auto cstep = [&](auto AL, auto KS, auto RH, auto MKc, auto WBc, float2 (&X)[8], float2 (&Yv)[8],
                     float& racc) __attribute__((always_inline)) {
      constexpr int ks = decltype(KS)::value;
      if constexpr (CS_REG_HOIST) {
        bool valid;
        int mode;
        const unsigned k2 = slot_k2(ks, valid, mode);   // recomputed: cheaper than a held register
        class_step<D2, M, decltype(RH)::value, decltype(MKc)::value, decltype(WBc)::value, decltype(AL)::value, TR>(
            X, Yv, rca[ks], rcb[ks], ryv[ks], k2, wk1, tp, a, racc);
      } else {
        float2 gca[D2], gcb[D2], gy;
        unsigned k2;
        load_ops(ks, gca, gcb, gy, k2);
        class_step<D2, M, decltype(RH)::value, decltype(MKc)::value, decltype(WBc)::value, decltype(AL)::value, TR>(
            X, Yv, gca, gcb, gy, k2, wk1, tp, a, racc);
      }
    };
    auto row_elem = [&](unsigned r) __attribute__((always_inline)) -> unsigned { return (wp * N2 + rt + r * Q) * 2; };

    // column-pass roles
    const bool cact = tid < CB * QC / 2;
    unsigned cc = tid % CB, cu = tid / CB;
    unsigned cjA = cu, cjB = cu ? QC - cu : QC / 2;
    unsigned j2c = j2_0 + cc;
    auto twc = [&](unsigned k1) __attribute__((always_inline)) -> float2 {   // W_N^{(j2 * k1) mod N}
      const unsigned ex = (j2c * k1) & (N - 1);
      return cmul(tlo[ex & ((1u << LOB) - 1)], thi[ex >> LOB]);
    };
    auto pair_elem = [&](unsigned w) __attribute__((always_inline)) -> unsigned { return (w * N2 + j2c) * 2; };
    // four-step twiddles of butterfly j's rows j + r*QC:
    // W_N^{j2 (j + r QC)} = W_N^{j2 j} * w^r with w = W_N^{j2 QC}; w^r from
    // w and w^4 by products (at most two), as in the FFT stages
    struct ColTw { float2 bA, bB, w1, w2, w3, w4; };
    auto col_tw = [&]() __attribute__((always_inline)) -> ColTw {
      ColTw c;
      c.bA = twc(cjA);
      c.bB = twc(cjB);
      c.w1 = twc(QC);
      c.w4 = twc(4 * QC);
      c.w2 = cmul(c.w1, c.w1);
      c.w3 = cmul(c.w2, c.w1);
      return c;
    };
    auto wpow = [&](const ColTw& c, int r) __attribute__((always_inline)) -> float2 {
      const float2 lo = (r & 3) == 1 ? c.w1 : ((r & 3) == 2 ? c.w2 : c.w3);
      if (r == 0) return c2(1.f, 0.f);
      if (r == 4) return c.w4;
      return r < 4 ? lo : cmul(c.w4, lo);
    };
    // Y entries of pairs cjA + r*QC and cjB + r*QC (r < 4) hold rows
    // k1 = cjA + r*QC, cjB + r*QC (side 0) and N1 - k1 (side 1); for cu > 0
    // the latter are butterfly cjB / cjA at 7 - r, for cu = 0 (butterflies 0
    // and QC/2, each its own mirror) they are the same butterfly at
    // (8 - r) mod 8 (r = 0: row N1/2, index 4) and 7 - r.
    auto col_load = [&](float2 (&A)[8], float2 (&B)[8]) __attribute__((always_inline)) {
      float2 lo[4], hi[4], lo2[4], hi2[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        ld_coh_pair(rs, pair_elem(cjA + r * QC), lo[r], hi[r]);
        ld_coh_pair(rs, pair_elem(cjB + r * QC), lo2[r], hi2[r]);
      }
      // every element is written at a fixed index with a value select of
      // opaque register values: stores at different indices in two branches,
      // or a select of two array loads, would become an access through a
      // selected address, which moves the arrays to scratch memory
      const ColTw ct = col_tw();
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        float2 h1 = hi[r], h2 = hi2[r], h3 = hi[(r + 1) & 3];
        opaque(h1); opaque(h2); opaque(h3);
        const float2 wl = wpow(ct, r), wh = wpow(ct, 7 - r);
        A[r] = cmulc(lo[r], cmul(ct.bA, wl));
        B[r] = cmulc(lo2[r], cmul(ct.bB, wl));
        A[7 - r] = cmulc(cu ? h2 : h3, cmul(ct.bA, wh));
        B[7 - r] = cmulc(cu ? h1 : h2, cmul(ct.bB, wh));
      }
    };
    auto col_store = [&](float2 (&A)[8], float2 (&B)[8]) __attribute__((always_inline)) {
      const ColTw ct = col_tw();
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        const float2 wr = wpow(ct, r);
        A[r] = cmul(A[r], cmul(ct.bA, wr));
        B[r] = cmul(B[r], cmul(ct.bB, wr));
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        float2 b7 = B[7 - r], a7 = A[7 - r], a8 = A[r == 0 ? 4 : 8 - r];
        opaque(b7); opaque(a7); opaque(a8);
        st_coh_pair(rs, pair_elem(cjA + r * QC), A[r], cu ? b7 : a8);
        st_coh_pair(rs, pair_elem(cjB + r * QC), B[r], cu ? a7 : b7);
      }
    };
    // forward column transform of (A, B) (time domain) and store to Y
    auto col_forward = [&](float2 (&A)[8], float2 (&B)[8]) __attribute__((always_inline)) {
      if (cact) {
        reg_stage_first<N1, CB, false, true, N1>(lds, A, cc, cjA);
        reg_stage_first<N1, CB, false, true, N1>(lds, B, cc, cjB);
      }
      __syncthreads();
      lds_fft_mid<N1, CB, T, false, true, N1>(lds, t1, tid);
      if (cact) {
        reg_stage_last<N1, CB, false, true, N1>(lds, t1, A, cc, cjA);
        reg_stage_last<N1, CB, false, true, N1>(lds, t1, B, cc, cjB);
        col_store(A, B);
      }
    };
    auto sidx = [&](unsigned j, unsigned r) __attribute__((always_inline)) -> unsigned { return (j + r * QC) * N2 + j2c; };

    // time-domain state of butterflies cjA, cjB (ISTA: x; ADMM: u)
    float2 stA[8], stB[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) { stA[r] = c2(0.f, 0.f); stB[r] = c2(0.f, 0.f); }
    unsigned nbar = 0;
    constexpr int NC = G < kBarCounters ? G : kBarCounters;
    constexpr unsigned PER_C = G / NC;

    if (ALG == 1 && a.warm) {
      const float2* z2 = reinterpret_cast<const float2*>(a.z);
      const float2* u2 = reinterpret_cast<const float2*>(a.u);
      float2 A[8], B[8];
      if (cact) {
#pragma unroll
        for (int r = 0; r < 8; ++r) {
          stA[r] = u2[sidx(cjA, r)];
          stB[r] = u2[sidx(cjB, r)];
          A[r] = csub(z2[sidx(cjA, r)], stA[r]);
          B[r] = csub(z2[sidx(cjB, r)], stB[r]);
        }
      }
      col_forward(A, B);
      grid_barrier<NC>(a.bar, (++nbar) * PER_C, a.err, a.max_ticks);
    }
    __syncthreads();

    for (int t = 1; t <= a.iters; ++t) {
      // recompute per-thread indices inside the iteration (hoisting them out
      // of the loop keeps dozens of addresses live and forces spills)
      asm volatile("" : "+v"(rpi), "+v"(rt), "+v"(wp), "+v"(jA), "+v"(jB), "+v"(sA), "+v"(sB));
      asm volatile("" : "+v"(cc), "+v"(cu), "+v"(cjA), "+v"(cjB), "+v"(j2c));
      // ---- row pass ----------------------------------------------------------
      float2 va[8], vb[8];
      const bool zero_in = (t == 1) && !(ALG == 1 && a.warm);
      if (ract) {
#pragma unroll
        for (int r = 0; r < 8; ++r) {
          if (zero_in) { va[r] = c2(0.f, 0.f); vb[r] = c2(0.f, 0.f); }
          else ld_coh_pair(rs, row_elem(r), va[r], vb[r]);
        }
        reg_stage_first<N2, RA, false, false, LDA>(lds, va, 2 * rpi, rt);
        reg_stage_first<N2, RA, false, false, LDA>(lds, vb, 2 * rpi + 1, rt);
      }
      __syncthreads();
      lds_fft_mid<N2, RA, T, false, false, LDA>(lds, t2, tid);
      if (ract) {
        reg_stage_last<N2, RA, false, false, LDA>(lds, t2, va, sA, jA);
        reg_stage_last<N2, RA, false, false, LDA>(lds, t2, vb, sB, jB);
      }
      __syncthreads();
      float racc = 0.0f;
      {
        using AL_ = std::integral_constant<int, ALG>;
        using std::integral_constant;
        using I0 = integral_constant<int, 0>;
        using I1 = integral_constant<int, 1>;
        using BT = std::true_type;
        using BF = std::false_type;
        if (cat == 0) {
          static_for<0, RM>([&](auto K) __attribute__((always_inline)) { cstep(AL_{}, K, K, I0{}, BT{}, va, vb, racc); });
        } else if (cat == 1 || cat == 3) {
          if constexpr (RM >= 2) {
            static_for<0, RM / 2>([&](auto K) __attribute__((always_inline)) {
              cstep(AL_{}, K, K, I0{}, BT{}, va, vb, racc);
              cstep(AL_{}, integral_constant<int, RM / 2 + decltype(K)::value>{}, K, I0{}, BT{}, vb, va, racc);
            });
          } else {
            cstep(AL_{}, I0{}, I0{}, I0{}, BT{}, va, vb, racc);
          }
        } else if (cat == 2) {
          if constexpr (RM >= 2) {
            static_for<0, RM / 2 + 1>([&](auto K) __attribute__((always_inline)) {
              constexpr int k = decltype(K)::value;
              cstep(AL_{}, K, K, I1{}, std::bool_constant<(k != 0 && k != RM / 2)>{}, va, va, racc);
            });
            static_for<0, RM / 2>([&](auto K) __attribute__((always_inline)) {
              cstep(AL_{}, integral_constant<int, RM / 2 + 1 + decltype(K)::value>{}, K, I0{}, BT{}, vb, vb, racc);
            });
          } else {
            cstep(AL_{}, I0{}, I0{}, I1{}, BF{}, va, va, racc);
            cstep(AL_{}, I1{}, I0{}, I0{}, BF{}, vb, vb, racc);
          }
        }
      }
      if (ract) {
        reg_stage_first<N2, RA, true, false, LDA>(lds, va, sA, jA);
        reg_stage_first<N2, RA, true, false, LDA>(lds, vb, sB, jB);
      }
      __syncthreads();
      lds_fft_mid<N2, RA, T, true, false, LDA>(lds, t2, tid);
      if (ract) {
        reg_stage_last<N2, RA, true, false, LDA>(lds, t2, va, 2 * rpi, rt);
        reg_stage_last<N2, RA, true, false, LDA>(lds, t2, vb, 2 * rpi + 1, rt);
#pragma unroll
        for (int r = 0; r < 8; ++r) st_coh_pair(rs, row_elem(r), va[r], vb[r]);
      }
      if constexpr (TR) {
        // ISTA: residual of x(t-1) (none at t = 1); ADMM: of the updated x(t)
        const double rs_ = block_sum<T>(double(racc), tid);
        if (tid == 0 && (ALG == 1 || t >= 2)) a.res[size_t(ALG == 1 ? t - 1 : t - 2) * G + g] = rs_;
      }
      grid_barrier<NC>(a.bar, (++nbar) * PER_C, a.err, a.max_ticks);

      // ---- column pass -------------------------------------------------------
      float2 A[8], B[8];
      if (cact) {
        col_load(A, B);
        reg_stage_first<N1, CB, true, true, N1>(lds, A, cc, cjA);
        reg_stage_first<N1, CB, true, true, N1>(lds, B, cc, cjB);
      }
      __syncthreads();
      lds_fft_mid<N1, CB, T, true, true, N1>(lds, t1, tid);
      if (cact) {
        reg_stage_last<N1, CB, true, true, N1>(lds, t1, A, cc, cjA);
        reg_stage_last<N1, CB, true, true, N1>(lds, t1, B, cc, cjB);
      }
      __syncthreads();
      const bool last = (t == a.iters);
      const float thr = a.thr;
      float l1acc = 0.0f;
      if (cact) {
        auto epi = [&](float2& v, float2& s, unsigned j, unsigned r) __attribute__((always_inline)) {
          if constexpr (ALG == 0) {
            const float2 w = cadd(s, v);
            const float2 xv = c2(soft(w.x, thr), soft(w.y, thr));
            if constexpr (TR) l1acc += fabsf(xv.x) + fabsf(xv.y);
            s = xv;
            v = xv;
          } else {
            const float2 xv = v;
            if constexpr (TR) l1acc += fabsf(xv.x) + fabsf(xv.y);
            const float2 xu = cadd(xv, s);
            const float2 zv = c2(soft(xu.x, thr), soft(xu.y, thr));
            const float2 u1 = csub(xu, zv);
            s = u1;
            if (last) {
              reinterpret_cast<float2*>(a.x)[sidx(j, r)] = xv;
              reinterpret_cast<float2*>(a.z)[sidx(j, r)] = zv;
            } else {
              v = csub(zv, u1);
            }
          }
        };
#pragma unroll
        for (int r = 0; r < 8; ++r) {
          epi(A[r], stA[r], cjA, r);
          epi(B[r], stB[r], cjB, r);
        }
      }
      if constexpr (TR) {
        const double l1_ = block_sum<T>(double(l1acc), tid);
        if (tid == 0) a.l1[size_t(t - 1) * G + g] = l1_;
      }
      // a traced ISTA also transforms x(T), for its residual below
      if (!last || (TR && ALG == 0)) {
        col_forward(A, B);
        grid_barrier<NC>(a.bar, (++nbar) * PER_C, a.err, a.max_ticks);
      }
    }

    if constexpr (TR && ALG == 0) {
      // residual of x(T): forward row transforms and the class residuals
      if (a.iters > 0) {
        asm volatile("" : "+v"(rpi), "+v"(rt), "+v"(wp), "+v"(jA), "+v"(jB), "+v"(sA), "+v"(sB));
        float2 va[8], vb[8];
        if (ract) {
#pragma unroll
          for (int r = 0; r < 8; ++r) ld_coh_pair(rs, row_elem(r), va[r], vb[r]);
          reg_stage_first<N2, RA, false, false, LDA>(lds, va, 2 * rpi, rt);
          reg_stage_first<N2, RA, false, false, LDA>(lds, vb, 2 * rpi + 1, rt);
        }
        __syncthreads();
        lds_fft_mid<N2, RA, T, false, false, LDA>(lds, t2, tid);
        if (ract) {
          reg_stage_last<N2, RA, false, false, LDA>(lds, t2, va, sA, jA);
          reg_stage_last<N2, RA, false, false, LDA>(lds, t2, vb, sB, jB);
        }
        __syncthreads();
        // the class dispatch of the iteration in residual-only mode
        float racc = 0.0f;
        {
          using AL_ = std::integral_constant<int, 2>;
          using std::integral_constant;
          using I0 = integral_constant<int, 0>;
          using I1 = integral_constant<int, 1>;
          using BT = std::true_type;
          using BF = std::false_type;
          if (cat == 0) {
            static_for<0, RM>([&](auto K) __attribute__((always_inline)) { cstep(AL_{}, K, K, I0{}, BT{}, va, vb, racc); });
          } else if (cat == 1 || cat == 3) {
            if constexpr (RM >= 2) {
              static_for<0, RM / 2>([&](auto K) __attribute__((always_inline)) {
                cstep(AL_{}, K, K, I0{}, BT{}, va, vb, racc);
                cstep(AL_{}, integral_constant<int, RM / 2 + decltype(K)::value>{}, K, I0{}, BT{}, vb, va, racc);
              });
            } else {
              cstep(AL_{}, I0{}, I0{}, I0{}, BT{}, va, vb, racc);
            }
          } else if (cat == 2) {
            if constexpr (RM >= 2) {
              static_for<0, RM / 2 + 1>([&](auto K) __attribute__((always_inline)) {
                constexpr int k = decltype(K)::value;
                cstep(AL_{}, K, K, I1{}, std::bool_constant<(k != 0 && k != RM / 2)>{}, va, va, racc);
              });
              static_for<0, RM / 2>([&](auto K) __attribute__((always_inline)) {
                cstep(AL_{}, integral_constant<int, RM / 2 + 1 + decltype(K)::value>{}, K, I0{}, BT{}, vb, vb, racc);
              });
            } else {
              cstep(AL_{}, I0{}, I0{}, I1{}, BF{}, va, va, racc);
              cstep(AL_{}, I1{}, I0{}, I0{}, BF{}, vb, vb, racc);
            }
          }
        }
        const double rs_ = block_sum<T>(double(racc), tid);
        if (tid == 0) a.res[size_t(a.iters - 1) * G + g] = rs_;
      }
    }

    // ---- outputs -----------------------------------------------------------
    float2* out = reinterpret_cast<float2*>(ALG == 0 ? a.x : a.u);
    if ((ALG == 0 || a.iters > 0) && cact) {
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        out[sidx(cjA, r)] = stA[r];
        out[sidx(cjB, r)] = stB[r];
      }
    }
  } else {
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
    grid_barrier<NC>(a.bar, (++nbar) * PER_C, a.err, a.max_ticks);
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
  // row pass, first half: the workgroup's row pairs from Y (zeros when
  // zero_in) into LDS, forward row transforms.  Every row load is issued
  // before the first LDS store.
  auto row_forward = [&](bool zero_in) {
    {
      float2 rv[EA];
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
  };
  for (int t = 1; t <= a.iters; ++t) {
    // keep per-thread index arithmetic inside the iteration: hoisting it out
    // of the loop keeps dozens of addresses live and forces spills
    asm volatile("" : "+v"(tid));
    // ---- row pass: forward rows, alias-class update, inverse rows ----------
    row_forward((t == 1) && !(ALG == 1 && a.warm));
    float racc = 0.0f;
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
        if constexpr (TR) racc += (write_b ? 2.0f : 1.0f) * cabs2(csub(gy[k], S));
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
        if constexpr (TR) {
          float2 s1 = c2(0.f, 0.f), s2 = c2(0.f, 0.f);
#pragma unroll
          for (int l = 0; l < D2; ++l) { s1 = cadd(s1, cmul(gca[k][l], Va[l])); s2 = cadd(s2, cmul(gcb[k][l], Vb[l])); }
          racc += (write_b ? 2.0f : 1.0f) * cabs2(csub(gy[k], cscale(cadd(s1, cconj(s2)), a.inv_d)));
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
    if constexpr (TR) {
      // ISTA: residual of x(t-1) (none at t = 1); ADMM: of the updated x(t)
      const double rs_ = block_sum<T>(double(racc), tid);
      if (tid == 0 && (ALG == 1 || t >= 2)) a.res[size_t(ALG == 1 ? t - 1 : t - 2) * G + g] = rs_;
    }
    grid_barrier<NC>(a.bar, (++nbar) * PER_C, a.err, a.max_ticks);

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
    float l1acc = 0.0f;
#pragma unroll
    for (int k = 0; k < EB; ++k) {
      const unsigned e = tid + k * T;
      if (FB || e < NEB) {
        if constexpr (ALG == 0) {
          const float2 v = cadd(st[k], lds[lp(e)]);
          const float2 xv = c2(soft(v.x, thr), soft(v.y, thr));
          if constexpr (TR) l1acc += fabsf(xv.x) + fabsf(xv.y);
          st[k] = xv;
          lds[lp(e)] = xv;
        } else {
          const float2 xv = lds[lp(e)];
          if constexpr (TR) l1acc += fabsf(xv.x) + fabsf(xv.y);
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
    if constexpr (TR) {
      const double l1_ = block_sum<T>(double(l1acc), tid);
      if (tid == 0) a.l1[size_t(t - 1) * G + g] = l1_;
    }
    // a traced ISTA also transforms x(T), for its residual below
    if (!last || (TR && ALG == 0)) {
      __syncthreads();
      col_forward_store();
      grid_barrier<NC>(a.bar, (++nbar) * PER_C, a.err, a.max_ticks);
    }
  }

  if constexpr (TR && ALG == 0) {
    // residual of x(T): forward row transforms and the class residuals
    if (a.iters > 0) {
      asm volatile("" : "+v"(tid));
      row_forward(false);
      float racc = 0.0f;
#pragma unroll
      for (int k = 0; k < GPT; ++k) {
        const unsigned q = tid + k * T;
        if (q >= (unsigned)ncls) continue;
        const Cls c = decode(q);
        const bool write_b = !(c.mode == 1 && (c.k2 == 0 || c.k2 == (M >> 1)));
        const float2 wk1 = a.twk1[c.rowa];
        float2 s1 = c2(0.f, 0.f), s2 = c2(0.f, 0.f);
#pragma unroll
        for (int l = 0; l < D2; ++l) {
          const int p = c.k2 + l * M;
          const int qq = (c.mode == 1) ? ((N2 - p) & (N2 - 1)) : (N2 - 1 - p);
          const float2 gw = cmul(wk1, tp[p]);
          const float2 za = lds[lpr(c.sa * LDA + p)];
          const float2 zbc = cconj(lds[lpr(c.sb * LDA + qq)]);
          const float2 P = cscale(cadd(za, zbc), 0.5f);
          const float2 Q = cscale(cmulmi(csub(za, zbc)), 0.5f);
          const float2 wq = cmul(gw, Q);
          s1 = cadd(s1, cmul(gca[k][l], cadd(P, wq)));
          s2 = cadd(s2, cmul(gcb[k][l], cconj(csub(P, wq))));
        }
        racc += (write_b ? 2.0f : 1.0f) * cabs2(csub(gy[k], cscale(cadd(s1, cconj(s2)), a.inv_d)));
      }
      const double rs_ = block_sum<T>(double(racc), tid);
      if (tid == 0) a.res[size_t(a.iters - 1) * G + g] = rs_;
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
}

}  // namespace cs
