// Batched ISTA (Alg. 1) / ADMM (Alg. 2) over many independent signals of
// different lengths and decimations, in one persistent launch.
//
// Every signal is solved with the plain solver's arithmetic: the four-step
// N = N1 * N2 FFT of the packed real signal, the alias-class update in the
// frequency domain (ISTA step, or ADMM's Woodbury x-update in residual form),
// the soft threshold (Eq. 4) and ADMM's z / u updates in the time domain.
// The work of one pass over the whole batch is a list of items:
//   - a row item (s, w) is the row pair {w, N1 - w} of signal s (the row pass:
//     forward row FFT, alias-class update, inverse row FFT);
//   - a column item (s, b) is the block of 8 columns [8b, 8b + 8) of signal s
//     (the column pass: inverse column FFT, the time-domain epilogue, forward
//     column FFT).
// The host assigns the items to workgroups once per batch: each workgroup
// takes items of one size class (length and decimation) only, so its code is
// compiled for that class, and each class gets a share of the workgroups in
// proportion to its estimated cost.  A workgroup always owns the same row and
// column items, in set-up and in every iteration.  One
// launch runs the set-up passes (c_hat = DFT_n(c), then the n-point spectrum
// of P^T y, whose first m bins are DFT_m(y)) and all iterations, with a
// grid barrier between passes: every signal advances one iteration per pair
// of passes, so all lengths share the GPU at once.
//
// Memory: per signal, the spectrum buffer Y (N complex) and the c_hat and
// y_hat tables (N + 1 complex each) live in library scratch; the iterate
// (ISTA x, ADMM u) is the caller's output array.  Y, which workgroups on
// different XCDs exchange, and the iterate, which its owner reads back in the
// next iteration, go through device-coherent accesses; a table is written and
// read only by the workgroup that owns its rows.
#pragma once
#include <stdint.h>

#include "solve_persistent.hpp"

namespace cs {

constexpr int kPBThreads = kThreads;   // 256 threads per workgroup
constexpr int kPBMinLogN = 9;          // N = n/2 = 2^9 .. 2^17, i.e. n = 2^10 .. 2^18
constexpr int kPBMaxLogN = 17;
constexpr int kPBMaxN1 = 256;          // four-step split of the largest length
constexpr int kPBMaxN2 = 512;
// Barrier area of a batched launch: the grid-barrier counters and error flag
// (kBarWords words), then the leave counter on a line of its own.
constexpr int kPBLeave = kBarWords;
constexpr int kPBBarWords = kBarWords + kBarStride;

// Four-step split of N = 2^L complex points (the plans' split): odd L gives
// N2 = 2 N1, even L gives N2 = 4 N1.
constexpr int pb_n1(int L) { return (L % 2) ? (1 << ((L - 1) / 2)) : (1 << (L / 2 - 1)); }
constexpr int pb_n2(int L) { return (1 << L) / pb_n1(L); }

// Item sizes.  A row item holds AI consecutive row pairs and a column item CBW
// adjacent columns, so that one item covers about kPBRowPts / kPBColPts
// complex points whatever the length: every item pays one global round trip
// and one set of FFT stages, so short rows and columns are taken many at a
// time.
#ifndef CS_PB_ROW_PTS
#define CS_PB_ROW_PTS 2048
#endif
#ifndef CS_PB_COL_PTS
#define CS_PB_COL_PTS 2048
#endif
constexpr int kPBRowPts = CS_PB_ROW_PTS;
constexpr int kPBColPts = CS_PB_COL_PTS;
constexpr int pb_min(int a, int b) { return a < b ? a : b; }
constexpr int pb_max(int a, int b) { return a > b ? a : b; }
constexpr int pb_ai(int L) { return pb_max(1, pb_min(pb_n1(L) / 2, kPBRowPts / (2 * pb_n2(L)))); }
// (the largest length, N1 = 256, takes 16 columns rather than 8: 128-byte
// runs of the spectrum and the iterate instead of 64-byte ones)
constexpr int pb_cbw(int L) {
  return L == kPBMaxLogN ? 16 : pb_max(kColsPerBlock, pb_min(pb_n2(L), kPBColPts / pb_n1(L)));
}
// LDS of one item: 2 AI rows of N2 (+ padding) or N1 x CBW interleaved
constexpr int kPBRowLds = lds_rows(kPBRowPts + 2 * kPBMaxN1 * kPadA);
constexpr int kPBColLds = lds_padded(pb_max(kPBColPts, kPBMaxN1 * 16));
constexpr int kPBLds = pb_max(kPBRowLds, kPBColLds);
// LDS copy of the four-step twiddles W_N^e (two levels) of the largest length
constexpr int kPBMaxTwN = (1 << ((kPBMaxLogN + 1) / 2)) + (1 << (kPBMaxLogN - (kPBMaxLogN + 1) / 2));

// One signal of the batch (built on the host).
struct PSig {
  float2* Y;               // scratch: N complex (four-step spectrum buffer)
  float2* chat;            // scratch: N + 1 complex, c_hat table
  float2* yhat;            // scratch: N + 1 complex, DFT_n(P^T y) table
  const float* c;          // generator, n
  const float* y;          // measurements, m
  float* x;                // ISTA: iterate and output; ADMM: output x
  float* z;                // ADMM: in (warm) / out
  float* u;                // ADMM: in (warm) / out, the scaled dual (state)
  const float* lam;        // device scalar lambda
  const float* par;        // device scalar: ISTA tau, ADMM rho
  const float2* twk1;      // W_n^{k1}
  const float2* twp;       // W_{2 N2}^p
  const float2* twlo;      // W_N^e, e < 2^lo_bits
  const float2* twhi;      // W_N^{e * 2^lo_bits}
  const float2* tw1;       // W_{N1}
  const float2* tw2;       // W_{N2}
  int logN;                // N = 2^logN
  int lo_bits;
  int d;                   // decimation (2, 4 or 8)
  int pad;
};

// One item of a pass: signal index and the first row pair w of its AI pairs
// (row pass) or the index b of its block of CBW columns (column pass).
struct PItem {
  unsigned sig;
  unsigned blk;
};

struct PBatchArgs {
  const PSig* sigs;
  const PItem* rows;       // row items, workgroup g's at [row_off[g], row_off[g+1])
  const PItem* cols;       // column items, likewise with col_off
  const unsigned* row_off;
  const unsigned* col_off;
  const unsigned* wg_class; // workgroup g's size class: (log2 N) << 4 | d/2
  unsigned* bar;           // barrier area (kPBBarWords words), counters zero at launch
  int* err;                // set to 1 if a barrier wait hit its bound
  uint64_t max_ticks;      // bound of one barrier wait in wall-clock ticks
  int iters;               // >= 1
  int warm;                // ADMM: start from the z, u passed in
};

// Grid barrier for any grid size G: workgroup g arrives on counter g mod NC
// (NC = min(G, kBarCounters), each on its own 128-byte line), so counter c
// receives G / NC + (c < G mod NC) arrivals per barrier; wave 0 polls every
// counter at once.  Waits are bounded as in grid_barrier.
__device__ __forceinline__ void pb_barrier(unsigned* bar, unsigned k, int* err, uint64_t max_ticks) {
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x < 64) {
    const unsigned G = gridDim.x;
    const unsigned NC = G < (unsigned)kBarCounters ? G : (unsigned)kBarCounters;
    const unsigned lane = threadIdx.x;
    if (lane == 0)
      __hip_atomic_fetch_add(bar + (blockIdx.x % NC) * kBarStride, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint64_t t0 = wall_clock64();
    while (true) {
      bool ok = true;
#pragma unroll
      for (unsigned c0 = 0; c0 < (unsigned)kBarCounters; c0 += 64) {
        const unsigned c = c0 + lane;
        if (c < NC) {
          const unsigned need = k * (G / NC + (c < G % NC ? 1u : 0u));
          ok &= __hip_atomic_load(bar + c * kBarStride, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= need;
        }
      }
      if (__all(ok)) break;
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

// Pass arguments of signal s (read from its descriptor).
__device__ __forceinline__ PassAArgs pb_row_args(const PSig& s, int alg) {
  const int L = s.logN;
  const int N1 = pb_n1(L);
  const int N = 1 << L;
  const int64_t n = int64_t(2) * N;
  PassAArgs a{};
  a.Y = s.Y;
  a.chat = s.chat;
  a.yhat = s.yhat;
  a.table = nullptr;
  a.tw2 = s.tw2;
  a.twk1 = s.twk1;
  a.twp = s.twp;
  a.N1 = N1;
  a.M = int((n / s.d) / N1);
  a.N = N;
  a.inv_n = 1.0f / float(n);
  a.inv_d = 1.0f / float(s.d);
  if (alg == 0) {
    a.tau = *s.par;
  } else {
    const float rho = *s.par;
    a.rho = rho;
    a.inv_rho = 1.0f / rho;
    a.d_rho = float(s.d) * rho;
  }
  return a;
}

__device__ __forceinline__ PassBArgs pb_col_args(const PSig& s, int alg) {
  const int L = s.logN;
  PassBArgs b{};
  b.Y = s.Y;
  b.tw1 = s.tw1;
  b.twlo = s.twlo;
  b.twhi = s.twhi;
  b.lo_bits = s.lo_bits;
  b.N2 = pb_n2(L);
  b.N = 1 << L;
  b.d = s.d;
  if (alg == 0) {
    b.u = s.x;
    b.thr = (*s.par) * (*s.lam);          // tau * lambda
  } else {
    b.u = s.u;
    b.thr = (*s.lam) / (*s.par);          // lambda / rho
    b.out0 = s.x;
    b.out1 = s.z;
  }
  return b;
}

// Zero (device-coherent stores) the CBW columns [CBW blk, CBW blk + CBW) of
// a time-domain array of N float2 laid out as [j1][N2].
template <int N1, int N2, int CBW>
__device__ __forceinline__ void pb_zero_cols(float* p, int blk) {
  const Gf2<true> q(reinterpret_cast<float2*>(p), unsigned(N1 * N2));
  for (int i = threadIdx.x; i < N1 * CBW; i += kPBThreads)
    q.st((size_t)(i / CBW) * N2 + blk * CBW + (i % CBW), c2(0.f, 0.f));
}

// Zero the rows of the AI pairs from w0 ({w, N1 - w}, {0, N1/2} for w = 0)
// of a spectrum buffer.
template <int N1, int N2, int AI>
__device__ __forceinline__ void pb_zero_rows(float2* Y, int w0) {
  const Gf2<true> q(Y, unsigned(N1 * N2));
  for (int i = threadIdx.x; i < 2 * AI * N2; i += kPBThreads) {
    const int slot = i / N2, w = w0 + (slot >> 1);
    const int row = (slot & 1) ? (w ? N1 - w : (N1 >> 1)) : w;
    q.st((size_t)row * N2 + (i % N2), c2(0.f, 0.f));
  }
}

// The whole solve for the items of one workgroup, all of one size class
// (length 2 * 2^L and decimation 2 * D2): set-up passes, iterations, with the
// grid barriers every workgroup of the launch takes in the same order.
// Not inlined: each size class's body gets a register allocation of its own
// (inlined together, the largest class's live ranges spill into every other).
template <int ALG, int L, int D2>
__device__ __noinline__ void pb_body(const PBatchArgs& a, float2* __restrict__ lds, float2* __restrict__ twr,
                                     float2* __restrict__ twc, float2* __restrict__ twn, unsigned& nbar) {
  constexpr int N1 = pb_n1(L), N2 = pb_n2(L);
  constexpr int AI = pb_ai(L), CBW = pb_cbw(L);
  static_assert((N1 / 2) % AI == 0 && N2 % CBW == 0, "item split");
  static_assert(lds_rows(2 * AI * (N2 + kPadA)) <= kPBLds && N1 * CBW <= kPBLds, "item exceeds the LDS buffer");
  constexpr int OPI = ALG == 0 ? A_ISTA : A_ADMM;
  constexpr int MODEI = ALG == 0 ? B_ISTA : B_ADMM;
  const int g = blockIdx.x;
  const unsigned r0 = a.row_off[g], r1 = a.row_off[g + 1];
  const unsigned c0 = a.col_off[g], c1 = a.col_off[g + 1];
  const unsigned tid = threadIdx.x;
  auto barrier = [&] { pb_barrier(a.bar, ++nbar, a.err, a.max_ticks); };

  // stage twiddles of this size class: W_{N2} (row pass), W_{N1} (column
  // pass) and the four-step W_N^e (two levels)
  constexpr int LO = (L + 1) / 2;
  if (r1 > r0 || c1 > c0) {
    const PSig& s0 = a.sigs[r1 > r0 ? a.rows[r0].sig : a.cols[c0].sig];
    for (int i = tid; i < N2; i += kPBThreads) twr[i] = s0.tw2[i];
    for (int i = tid; i < N1; i += kPBThreads) twc[i] = s0.tw1[i];
    for (int i = tid; i < (1 << LO); i += kPBThreads) twn[i] = s0.twlo[i];
    for (int i = tid; i < (1 << (L - LO)); i += kPBThreads) twn[(1 << LO) + i] = s0.twhi[i];
  }
  // Each item recomputes its per-thread indices from a thread index the
  // compiler cannot see through: hoisted out of the loops, the index and
  // address arithmetic of every pass stays live across all of them and
  // spills.
  auto lane_id = [&] {
    unsigned t = tid;
    asm volatile("" : "+v"(t));
    return t;
  };
  auto rows = [&](auto&& f) {
    for (unsigned it = r0; it < r1; ++it) {
      const PItem item = a.rows[it];
      const PSig& s = a.sigs[item.sig];
      __syncthreads();
      f(s, int(item.blk), lane_id());
    }
  };
  auto cols = [&](auto&& f) {
    for (unsigned it = c0; it < c1; ++it) {
      const PItem item = a.cols[it];
      const PSig& s = a.sigs[item.sig];
      __syncthreads();
      f(s, int(item.blk), lane_id());
    }
  };

  // ---- set-up: c_hat, then the spectrum of P^T y; initial state ----------
  cols([&](const PSig& s, int blk, unsigned tq) {
    PassBArgs b = pb_col_args(s, ALG);
    b.in0 = s.c;
    colpass<N1, B_FWD_REAL, kPBThreads, true, CBW, true>(b, blk, lds, twc, tq, twn);
  });
  barrier();
  rows([&](const PSig& s, int w, unsigned tq) {
    PassAArgs ra = pb_row_args(s, ALG);
    ra.table = s.chat;
    rowpass<N2, A_SPEC, D2, kPBThreads, true, AI>(ra, w, lds, twr, tq);
  });
  barrier();
  cols([&](const PSig& s, int blk, unsigned tq) {
    PassBArgs b = pb_col_args(s, ALG);
    b.in0 = s.y;
    colpass<N1, B_FWD_UP, kPBThreads, true, CBW, true>(b, blk, lds, twc, tq, twn);
  });
  barrier();
  // The first iteration starts from x = 0 (ISTA) or z = u = 0 (cold ADMM):
  // a zero spectrum and a zero state.
  const bool zero = (ALG == 0) || !a.warm;
  rows([&](const PSig& s, int w, unsigned tq) {
    PassAArgs ra = pb_row_args(s, ALG);
    ra.table = s.yhat;
    rowpass<N2, A_SPEC, D2, kPBThreads, true, AI>(ra, w, lds, twr, tq);
    if (zero) {
      __syncthreads();
      pb_zero_rows<N1, N2, AI>(s.Y, w);
    }
  });
  if (zero) {
    cols([&](const PSig& s, int blk, unsigned) { pb_zero_cols<N1, N2, CBW>(ALG == 0 ? s.x : s.u, blk); });
  }
  barrier();
  if constexpr (ALG == 1) {
    if (a.warm) {
      // warm start: Y = forward transform of z - u
      cols([&](const PSig& s, int blk, unsigned tq) {
        PassBArgs b = pb_col_args(s, ALG);
        b.in0 = s.z;
        b.in1 = s.u;
        colpass<N1, B_FWD_ZMU, kPBThreads, true, CBW, true>(b, blk, lds, twc, tq, twn);
      });
      barrier();
    }
  }

  // ---- iterations ---------------------------------------------------------
  // The last iteration is written out separately so that `last` is a
  // compile-time constant in each column-pass instance.
  auto iteration = [&](auto last_c) {
    rows([&](const PSig& s, int w, unsigned tq) {
      const PassAArgs ra = pb_row_args(s, ALG);
      rowpass<N2, OPI, D2, kPBThreads, true, AI>(ra, w, lds, twr, tq);
    });
    barrier();
    cols([&](const PSig& s, int blk, unsigned tq) {
      PassBArgs b = pb_col_args(s, ALG);
      b.last = decltype(last_c)::value;
      colpass<N1, MODEI, kPBThreads, true, CBW, true>(b, blk, lds, twc, tq, twn);
    });
  };
  for (int t = 1; t < a.iters; ++t) {
    iteration(std::integral_constant<int, 0>{});
    barrier();
  }
  iteration(std::integral_constant<int, 1>{});
}

template <int ALG, int L>
__device__ __forceinline__ void pb_body_d(const PBatchArgs& a, int d2, float2* lds, float2* twr, float2* twc,
                                          float2* twn, unsigned& nbar) {
  if (d2 == 1) pb_body<ALG, L, 1>(a, lds, twr, twc, twn, nbar);
  else if (d2 == 2) pb_body<ALG, L, 2>(a, lds, twr, twc, twn, nbar);
  else pb_body<ALG, L, 4>(a, lds, twr, twc, twn, nbar);
}

template <int ALG>   // 0: ISTA, 1: ADMM
__global__ __launch_bounds__(kPBThreads, 3) void k_batch_persist(PBatchArgs a) {
  __shared__ float2 lds[kPBLds];
  __shared__ float2 twr[kPBMaxN2];
  __shared__ float2 twc[kPBMaxN1];
  __shared__ float2 twn[kPBMaxTwN];
  unsigned nbar = 0;
  // this workgroup's size class: length 2^(L+1), decimation 2 * d2
  const unsigned cls = a.wg_class[blockIdx.x];
  const int L = int(cls >> 4), d2 = int(cls & 15);
  switch (L) {
    case 9: pb_body_d<ALG, 9>(a, d2, lds, twr, twc, twn, nbar); break;
    case 10: pb_body_d<ALG, 10>(a, d2, lds, twr, twc, twn, nbar); break;
    case 11: pb_body_d<ALG, 11>(a, d2, lds, twr, twc, twn, nbar); break;
    case 12: pb_body_d<ALG, 12>(a, d2, lds, twr, twc, twn, nbar); break;
    case 13: pb_body_d<ALG, 13>(a, d2, lds, twr, twc, twn, nbar); break;
    case 14: pb_body_d<ALG, 14>(a, d2, lds, twr, twc, twn, nbar); break;
    case 15: pb_body_d<ALG, 15>(a, d2, lds, twr, twc, twn, nbar); break;
    case 16: pb_body_d<ALG, 16>(a, d2, lds, twr, twc, twn, nbar); break;
    default: pb_body_d<ALG, 17>(a, d2, lds, twr, twc, twn, nbar); break;
  }

  // ---- leave ----------------------------------------------------------------
  // The last workgroup to leave (every other one has passed every barrier by
  // then) sets the barrier counters and the leave counter back to zero, so the
  // next launch on the stream starts from zero without a separate clearing
  // step.
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x < 64) {
    unsigned old = 0;
    if (threadIdx.x == 0)
      old = __hip_atomic_fetch_add(a.bar + kPBLeave, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    old = __shfl(old, 0);
    if (old == gridDim.x - 1) {
      for (unsigned c = threadIdx.x; c < (unsigned)kBarCounters; c += 64)
        __hip_atomic_store(a.bar + c * kBarStride, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (threadIdx.x == 0) __hip_atomic_store(a.bar + kPBLeave, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

}  // namespace cs
