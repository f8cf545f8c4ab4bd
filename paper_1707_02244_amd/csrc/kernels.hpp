// Kernels of the partial-circulant LASSO path (ISTA, Alg. 1; ADMM, Alg. 2).
//
// Every product with A = P C or A^T goes through the DFT (circulants are
// diagonalised by the Fourier matrix, Section 4.2).  A length-n real signal x
// is packed as the complex sequence z_j = x_{2j} + i x_{2j+1}, j < N = n/2,
// and transformed with a four-step FFT N = N1 * N2:
//
//   pass B ("columns", this file's k_passB): for each column j2, an N1-point
//     FFT over j1 of z[N2*j1 + j2], times W_N^{j2*k1}; stored as Y[k1][j2].
//   pass A ("rows", k_passA): for a row k1, an N2-point FFT over j2 gives the
//     packed spectrum Z at bins k = k1 + N1*k2 in position k2.
//
// The real spectrum follows from Z by the usual split
//   X_k = P + W_n^k Q,  X_{N-k} = conj(P - W_n^k Q),
//   P = (Z_k + conj Z_{N-k})/2,  Q = -i (Z_k - conj Z_{N-k})/2,
// and bins k and N-k sit in rows k1 and N1-k1.  Decimation by d (P keeps every
// d-th sample) aliases the n-point spectrum onto m = n/d bins: the m-point
// spectrum of P w is (1/d) sum_l W_{k'+l m}.  When N1 divides m, the d bins
// of an alias class lie in rows k1 and N1-k1 too, so one workgroup owning that
// row pair sees every bin its frequency-domain update touches.
//
// The frequency-domain updates (per alias class k', with a = the class's
// bins in [0, N), b = the mirrored bins N - k'- l m, S = A x in the m-point
// domain, c_hat = DFT_n(c), Y_hat = DFT_m(y)):
//   ISTA (Alg. 1 with the tau*lam threshold):
//     S = (sum_a c_a X_a + conj(sum_b c_b X_b)) / d,  E = Y_hat - S,
//     D_a = tau conj(c_a) E,  D_b = tau conj(c_b) conj(E)   (= DFT of tau A^T r)
//     x+ = eta_{tau lam}(x + IDFT_n D)
//   The iterate x stays in the time domain and only the step tau A^T r
//   goes through the inverse transform: carrying x itself through a forward
//   and inverse FP32 FFT every iteration adds round-off that accumulates
//   along ISTA's slowly contracting directions.
//   ADMM x-update (Alg. 2, with (A^T A + rho I)^{-1} applied by Woodbury:
//     (A^T A + rho I)^{-1} = rho^{-1}[I - A^T (rho I + A A^T)^{-1} A], and
//     A A^T is the m x m circulant with eigenvalues
//     Lam_k' = (1/d) sum_class |c_hat|^2).  With Q_a = conj(c_a) Y_hat +
//     rho X_a (X: the spectrum of z - u) the Woodbury form is
//     X'_a = (Q_a - conj(c_a) T)/rho, T = (sum c_a Q_a + conj sum c_b Q_b) /
//     (d rho + sum |c|^2); substituting Q gives the residual form used here,
//     X'_a = X_a + conj(c_a) E,  X'_b = X_b + conj(c_b) conj(E),
//     E = d (Y_hat - S) / (d rho + sum |c|^2),
//   which avoids subtracting two nearly equal terms when Lam >> rho.
// The time-domain steps (soft threshold, Eq. 4; ADMM's z and u updates) are
// fused into pass B between its inverse and forward column transforms.
#pragma once
#include "cplx.hpp"
#include "fft_lds.hpp"

namespace cs {

constexpr int kThreads = 256;
// Threads of the two-launch row and column passes: 256, more for the long
// rows and columns of n >= 2^23 (2 x 4096-point rows, 1024- to 4096-point
// columns in blocks of 8 or 4), whose single workgroup per CU would
// otherwise hold 4 waves.
#ifndef CS_PASS_WIDE
#define CS_PASS_WIDE 1
#endif
constexpr int pass_a_threads(int N2) { return CS_PASS_WIDE && N2 >= 8192 ? 1024 : (CS_PASS_WIDE && N2 >= 4096 ? 512 : kThreads); }
constexpr int pass_b_threads(int N1) { return CS_PASS_WIDE && N1 >= 2048 ? 1024 : (CS_PASS_WIDE && N1 >= 1024 ? 512 : kThreads); }
constexpr int kColsPerBlock = 8;   // pass B: adjacent columns per workgroup (64 B runs)
constexpr int kPadA = CS_ROW_PAD ? 0 : 4;   // pass A: float2 padding between rows

enum OpA : int {
  A_ISTA = 0,   // ISTA frequency update (alias classes)
  A_ADMM = 1,   // ADMM Woodbury x-update (alias classes)
  A_MUL = 2,    // multiply by c_hat      (C x)
  A_MULC = 3,   // multiply by conj(c_hat) (C^T x)
  A_SPEC = 4,   // write the half spectrum X_k, k in [0, N], to a table
  A_ADJ = 5,    // adjoint step: S = A v (m-point spectrum), ybar += tau S,
                //   output -tau A^T A v   (the ISTA update with y = 0)
  A_TILE = 6,   // output the n-point spectrum of P^T r from r's m-point
                //   spectrum (the table in `ybar`)
  A_RES = 7,    // objective trace only: sum |Y_hat - S|^2 of the current
                //   iterate, no update
};

enum ModeB : int {
  B_FWD_REAL = 0,  // load real x (n)                 -> forward -> Y
  B_FWD_UP = 1,    // load P^T r (r has m = n/d)      -> forward -> Y
  B_FWD_ZMU = 2,   // load z - u (n each)             -> forward -> Y
  B_ISTA = 3,      // Y (step) -> inverse -> x += step, threshold -> forward -> Y
  B_ADMM = 4,      // Y -> inverse -> z, u update -> forward(z - u) -> Y (or write x, z)
  B_OUT_ALL = 5,   // Y -> inverse -> write all n reals
  B_OUT_DEC = 6,   // Y -> inverse -> write every d-th real (m values)
  B_ISTA_REC = 7,  // B_ISTA that also records v_t = x + step and the step
  B_ADJ_V = 8,     // xbar -> vbar = M_t * xbar, partial sums -> forward -> Y
  B_ADJ_X = 9,     // Y -> inverse -> xbar = vbar + (-tau A^T A vbar)
  B_ADJ_XV = 10,   // B_ADJ_X of step t fused with B_ADJ_V of step t-1: xbar_{t-1}
                   //   stays in registers (a.t, rv, rd, part are step t-1's)
};

struct PassAArgs {
  float2* Y;               // [N1][N2] workspace (in and out)
  const float2* chat;      // c_hat, bin k1 + N1*k2 at [k1*N2 + k2], Nyquist at [N]
  const float2* yhat;      // DFT_n(P^T y) in the same layout (= Y_hat at k' < m)
  float2* table;           // A_SPEC destination, same layout
  const float2* tw2;       // W_{N2}^e, e < N2
  const float2* twk1;      // W_n^{k1}, k1 < N1
  const float2* twp;       // W_{2 N2}^p, p < N2   (W_n^{N1 p})
  int N1;
  int M;                   // m / N1: alias classes per row
  int N;                   // N1 * N2
  float inv_n;             // 1/n
  float inv_d;             // 1/d
  float tau;               // ISTA step
  float rho, inv_rho, d_rho;
  const float* tau_dev;    // per-iteration steps (unrolled ISTA); used when set
  int t;                   // iteration index into tau_dev
  float2* ybar;            // A_ADJ: accumulated m-point spectrum; A_TILE: source
  double* res;             // objective trace (A_ISTA, A_ADMM, A_RES; when set):
                           //   res[w] = sum over workgroup w's m-point bins of
                           //   |Y_hat - S|^2, S = DFT_m(A x) of the iterate
                           //   (ISTA: the input x; ADMM: the updated x)
};

struct PassBArgs {
  float2* Y;               // [N1][N2] workspace
  const float2* tw1;       // W_{N1}^e, e < N1
  const float2* twlo;      // W_N^e, e < 2^lo_bits
  const float2* twhi;      // W_N^{e * 2^lo_bits}, e < N >> lo_bits
  int lo_bits;
  int N2;
  int N;
  int d;
  const float* in0;        // B_FWD_REAL: x; B_FWD_UP: r; B_FWD_ZMU: z
  const float* in1;        // B_FWD_ZMU: u
  float* out0;             // B_ADMM last: x; B_OUT_*: output
  float* out1;             // B_ADMM last: z
  float* u;                // state (n), read and written: B_ISTA x, B_ADMM u
  float thr;               // threshold (ISTA: tau*lam; ADMM: lam/rho)
  int last;                // final iteration: write outputs, skip the forward
  const float* tau_dev;    // per-iteration parameters (unrolled ISTA): the
  const float* lam_dev;    //   threshold is tau_dev[t] * lam_dev[t] when set
  int t;
  float* rv;               // B_ISTA_REC: v_t out; B_ADJ_V: v_t in
  float* rd;               // B_ISTA_REC: step out; B_ADJ_V: step in
  float* xbar;             // B_ADJ_V: in; B_ADJ_X: out
  float* vbar;             // B_ADJ_V: out; B_ADJ_X: in
  double* part;            // B_ADJ_V: per-workgroup partial sums (2 values)
  int part_q;              //   stride between the two sums
  double* l1;              // objective trace (B_ISTA, B_ADMM; when set):
                           //   l1[b] = sum of |x| over workgroup b's samples
};

// Data that workgroups of one persistent launch exchange (the spectrum
// buffer, and state a workgroup reads back in later iterations) is read and
// written with relaxed agent-scope atomic accesses: on gfx950 these are
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

// Buffer accesses with the device-coherence cache bit (sc1): the same
// coherence as the relaxed agent-scope atomics above, but as ordinary vector
// memory instructions that the compiler issues back to back (the atomic forms
// are kept in program order, one round trip each).  The resource covers the
// array exactly, so an offset outside it reads zeros and drops the store.
typedef unsigned cs_u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned cs_u32x4 __attribute__((ext_vector_type(4)));
constexpr int kCohAux = 16;                  // cache policy: sc1
constexpr int kBufWord3 = 0x00020000;        // raw 32-bit buffer (gfx9 family)

// Global float2 array access of the pass bodies: plain (COH = false, the
// launch-per-pass kernels, where kernel boundaries order everything) or
// device-coherent (persistent launches, whose workgroups exchange data
// within one launch).  `count` is the array's length in float2.
template <bool COH>
struct Gf2 {
  float2* p;
  __device__ __forceinline__ Gf2(float2* base, unsigned) : p(base) {}
  __device__ __forceinline__ float2 ld(size_t i) const { return p[i]; }
  __device__ __forceinline__ void st(size_t i, float2 v) const { p[i] = v; }
};
template <>
struct Gf2<true> {
  __amdgpu_buffer_rsrc_t rs;
  __device__ __forceinline__ Gf2(float2* base, unsigned count)
      : rs(__builtin_amdgcn_make_buffer_rsrc(base, 0, (int)(count * 8u), kBufWord3)) {}
  __device__ __forceinline__ float2 ld(size_t i) const {
    const cs_u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(rs, (unsigned)i * 8u, 0, kCohAux);
    return c2(__uint_as_float(v.x), __uint_as_float(v.y));
  }
  __device__ __forceinline__ void st(size_t i, float2 v) const {
    const cs_u32x2 w = {__float_as_uint(v.x), __float_as_uint(v.y)};
    __builtin_amdgcn_raw_buffer_store_b64(w, rs, (unsigned)i * 8u, 0, kCohAux);
  }
};

// Sum of v over the workgroup, returned to thread 0 (all threads call it).
template <int T>
__device__ __forceinline__ double block_sum(double v, unsigned tid) {
  __shared__ double red[T / 64];
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  if ((tid & 63) == 0) red[tid >> 6] = v;
  __syncthreads();
  double r = 0.0;
  if (tid == 0)
    for (int w = 0; w < T / 64; ++w) r += red[w];
  __syncthreads();
  return r;
}

// ---------------------------------------------------------------------------
// Four-step twiddle W_N^e from a two-level table.
__device__ __forceinline__ float2 tw_N(const PassBArgs& a, int e) {
  e &= (a.N - 1);
  return cmul(a.twlo[e & ((1 << a.lo_bits) - 1)], a.twhi[e >> a.lo_bits]);
}

// ---------------------------------------------------------------------------
// Pass A.  Workgroup w owns rows {w, N1 - w}; workgroup 0 owns the two rows
// that are their own mirror images, {0, N1/2}.  Rows are held in LDS slots 0
// and 1.  D2 = d/2 bins per alias-class side; D2 = 0 stands for d = 1
// (m = n): every bin is its own class, and A_ISTA, A_ADMM and A_RES run on
// the split pairs (k, N - k) with y_hat read at both bins.  LATE: load the
// class operands after the forward row transforms instead of with the rows
// (fewer registers live across the transforms).
template <int N2, int OP, int D2, int T, bool COH = false, int AI = 1, bool LATE = false>
__device__ __forceinline__ void rowpass(const PassAArgs& a, int w0, float2* __restrict__ lds,
                                        const float2* __restrict__ tws, unsigned tid) {
  constexpr int LD = N2 + kPadA;
  constexpr int NR = 2 * AI * N2;                     // elements of the held rows
  constexpr int EPT = (NR + T - 1) / T;               // row elements per thread
  constexpr bool SINGLE = (D2 == 0);                  // d = 1: single-bin classes
  static_assert(!SINGLE || OP == A_ISTA || OP == A_ADMM || OP == A_RES || OP == A_MUL || OP == A_MULC ||
                OP == A_SPEC, "single-bin classes: solver and operator modes only");
  constexpr bool GROUP = !SINGLE && (OP == A_ISTA || OP == A_ADMM || OP == A_ADJ || OP == A_TILE || OP == A_RES);
  constexpr bool NEED_C = (OP == A_ISTA || OP == A_ADMM || OP == A_ADJ || OP == A_RES);
  constexpr bool HAS_RES = (OP == A_ISTA || OP == A_ADMM || OP == A_RES);
  constexpr int DA = SINGLE ? 1 : D2;                 // array extent
  constexpr int MC = N2 / DA;                         // alias classes per row (= m / N1)
  constexpr int GPT = GROUP ? (AI * MC + 1 + T - 1) / T : 1;
  const int N1 = a.N1;
  const float tau = a.tau_dev ? a.tau_dev[a.t] : a.tau;
  // AI consecutive row pairs from w0: LDS slot 2i holds row w = w0 + i, slot
  // 2i + 1 its mirror N1 - w (N1/2 for w = 0)
  auto row_of = [&](int slot) {
    const int w = w0 + (slot >> 1);
    return (slot & 1) ? (w ? N1 - w : (N1 >> 1)) : w;
  };
  // item g of a per-pair range of `span` entries (span + 1 for pair 0):
  // its pair index pi and its index lc within the pair
  auto split_item = [&](int g, int span, int& pi, int& lc) {
    if (w0 == 0 && g <= span) { pi = 0; lc = g; }
    else if (w0 == 0) { pi = 1 + (g - span - 1) / span; lc = (g - span - 1) % span; }
    else { pi = g / span; lc = g % span; }
  };
  const Gf2<COH> Yg(a.Y, (unsigned)a.N);

  // Issue every global load before the first wait: the two rows and (update
  // modes) each class's c_hat, y_hat and split twiddles.
  float2 rv[EPT];
#pragma unroll
  for (int k = 0; k < EPT; ++k) {
    const int i = tid + k * T;
    if (NR % T == 0 || i < NR) {
      const int s = i / N2, p = i % N2;
      rv[k] = Yg.ld((size_t)row_of(s) * N2 + p);
    }
  }
  // class decode: mode 0 = row pair (w > 0); 1 = row 0; 2 = row N1/2 (w = 0)
  float2 gca[GPT][DA], gcb[GPT][DA], gw[GPT][DA], gy[GPT];
  const int M = MC;
  const int ng = (w0 ? M : (M + 1)) + (AI - 1) * M;   // classes of the held pairs
  auto load_classes = [&]() __attribute__((always_inline)) {
#pragma unroll
    for (int k = 0; k < GPT; ++k) {
      const int gi = tid + k * T;
      if (gi < ng) {
        int pi, g;
        split_item(gi, M, pi, g);
        const int w = w0 + pi;
        int rowa, k2, mode;
        if (w) { rowa = w; k2 = g; mode = 0; }
        else if (g <= (M >> 1)) { rowa = 0; k2 = g; mode = 1; }
        else { rowa = N1 >> 1; k2 = g - (M >> 1) - 1; mode = 2; }
        const int rowb = (mode == 0) ? (N1 - w) : rowa;
        const float2 wk1 = a.twk1[rowa];
#pragma unroll
        for (int l = 0; l < D2; ++l) {
          const int p = k2 + l * M;
          const int q = (mode == 1) ? ((N2 - p) & (N2 - 1)) : (N2 - 1 - p);
          gw[k][l] = cmul(wk1, a.twp[p]);
          if constexpr (NEED_C) {
            gca[k][l] = a.chat[(size_t)rowa * N2 + p];
            gcb[k][l] = (mode == 1 && p == 0) ? a.chat[a.N] : a.chat[(size_t)rowb * N2 + q];
          }
        }
        if constexpr (OP == A_ISTA || OP == A_ADMM || OP == A_RES) gy[k] = a.yhat[(size_t)rowa * N2 + k2];
        else if constexpr (OP == A_TILE) gy[k] = a.ybar[(size_t)rowa * N2 + k2];
      }
    }
  };
  if constexpr (GROUP && !LATE) load_classes();
#pragma unroll
  for (int k = 0; k < EPT; ++k) {
    const int i = tid + k * T;
    if (NR % T == 0 || i < NR) lds[lpr((i / N2) * LD + (i % N2))] = rv[k];
  }
  __syncthreads();
  lds_fft<N2, 2 * AI, T, false, false, LD>(lds, tws, tid);
  if constexpr (GROUP && LATE) load_classes();

  // objective trace: this thread's sum of weight * |Y_hat - S|^2; a class
  // stands for m-point bins k' and m - k' (weight 2) unless k' is 0 or m/2
  float res_acc = 0.0f;
  if constexpr (GROUP) {
    // Alias classes.  For w > 0: class k' = w + N1*k2, k2 < M, has a-bins at
    // row w positions k2 + l*M and b-bins at row N1-w positions N2-1-k2-l*M.
    // For w = 0: row 0 classes k2 in [0, M/2] (b positions (N2 - p) mod N2;
    // k2 = 0 and M/2 are their own mirror: write the a side only), then row
    // N1/2 classes k2 in [0, M/2) (b positions N2-1-p in the same row).
#pragma unroll
    for (int k = 0; k < GPT; ++k) {
      const int gi = tid + k * T;
      if (gi >= ng) continue;
      int pi, g;
      split_item(gi, M, pi, g);
      const int w = w0 + pi;
      int sa, sb, k2, mode;
      if (w) { sa = 2 * pi; sb = 2 * pi + 1; k2 = g; mode = 0; }
      else if (g <= (M >> 1)) { sa = 2 * pi; sb = 2 * pi; k2 = g; mode = 1; }
      else { sa = 2 * pi + 1; sb = 2 * pi + 1; k2 = g - (M >> 1) - 1; mode = 2; }
      const bool write_b = !(mode == 1 && (k2 == 0 || k2 == (M >> 1)));
      const float res_w = write_b ? 2.0f : 1.0f;
      float2 Xa[D2], Xb[D2];
      int pa[D2], qb[D2];
#pragma unroll
      for (int l = 0; l < D2; ++l) {
        const int p = k2 + l * M;
        const int q = (mode == 1) ? ((N2 - p) & (N2 - 1)) : (N2 - 1 - p);
        pa[l] = p; qb[l] = q;
        const float2 za = lds[lpr(sa * LD + p)];
        const float2 zbc = cconj(lds[lpr(sb * LD + q)]);
        const float2 P = cscale(cadd(za, zbc), 0.5f);
        const float2 Q = cscale(cmulmi(csub(za, zbc)), 0.5f);
        const float2 wq = cmul(gw[k][l], Q);
        Xa[l] = cadd(P, wq);
        Xb[l] = cconj(csub(P, wq));
      }
      float2 Va[D2], Vb[D2];
      if constexpr (OP == A_RES) {
        float2 sa_ = c2(0.f, 0.f), sb_ = c2(0.f, 0.f);
#pragma unroll
        for (int l = 0; l < D2; ++l) { sa_ = cadd(sa_, cmul(gca[k][l], Xa[l])); sb_ = cadd(sb_, cmul(gcb[k][l], Xb[l])); }
        const float2 S = cscale(cadd(sa_, cconj(sb_)), a.inv_d);
        res_acc += res_w * cabs2(csub(gy[k], S));
        continue;
      } else if constexpr (OP == A_ISTA || OP == A_ADJ) {
        // S = A x in the m-point domain; ISTA: tau A^T (y - A x);
        // adjoint: -tau A^T A x, and tau A x accumulated into ybar
        float2 sa_ = c2(0.f, 0.f), sb_ = c2(0.f, 0.f);
#pragma unroll
        for (int l = 0; l < D2; ++l) { sa_ = cadd(sa_, cmul(gca[k][l], Xa[l])); sb_ = cadd(sb_, cmul(gcb[k][l], Xb[l])); }
        const float2 S = cscale(cadd(sa_, cconj(sb_)), a.inv_d);
        float2 E;
        if constexpr (OP == A_ISTA) {
          const float2 r = csub(gy[k], S);
          res_acc += res_w * cabs2(r);
          E = cscale(r, tau);
        } else {
          E = cscale(S, -tau);
          const int rowa = w ? w : (mode == 1 ? 0 : (N1 >> 1));
          float2* yb = a.ybar + (size_t)rowa * N2 + k2;
          *yb = cadd(*yb, cscale(S, tau));
        }
        const float2 Ec = cconj(E);
#pragma unroll
        for (int l = 0; l < D2; ++l) {
          Va[l] = cconjmul(gca[k][l], E);
          Vb[l] = cconjmul(gcb[k][l], Ec);
        }
      } else if constexpr (OP == A_TILE) {
        // the n-point spectrum of P^T r is r's m-point spectrum repeated over
        // the d bins of each alias class (conjugated on the mirrored bins)
        const float2 r = gy[k], rc = cconj(gy[k]);
#pragma unroll
        for (int l = 0; l < D2; ++l) { Va[l] = r; Vb[l] = rc; }
      } else {
        // residual form of the Woodbury x-update (equal to (Q - conj(c) T) / rho):
        // X' = X + conj(c) E, E = d (Y_hat - S) / (d rho + sum |c|^2)
        const float2 yk = gy[k];
        float2 ra_ = c2(0.f, 0.f), rb_ = c2(0.f, 0.f);
        float den = a.d_rho;   // d*rho + sum over the class of |c_hat|^2 = d (rho + Lam)
#pragma unroll
        for (int l = 0; l < D2; ++l) {
          ra_ = cadd(ra_, cmul(gca[k][l], Xa[l]));
          rb_ = cadd(rb_, cmul(gcb[k][l], Xb[l]));
          den += cabs2(gca[k][l]) + cabs2(gcb[k][l]);
        }
        const float2 S = cscale(cadd(ra_, cconj(rb_)), a.inv_d);
        const float2 E = cscale(csub(yk, S), 1.0f / (den * a.inv_d));
        const float2 Ec = cconj(E);
#pragma unroll
        for (int l = 0; l < D2; ++l) {
          Va[l] = cadd(Xa[l], cconjmul(gca[k][l], E));
          Vb[l] = cadd(Xb[l], cconjmul(gcb[k][l], Ec));
        }
        if (a.res) {
          // residual of the updated x: S' = (sum c_a X'_a + conj sum c_b X'_b) / d
          float2 s1 = c2(0.f, 0.f), s2 = c2(0.f, 0.f);
#pragma unroll
          for (int l = 0; l < D2; ++l) { s1 = cadd(s1, cmul(gca[k][l], Va[l])); s2 = cadd(s2, cmul(gcb[k][l], Vb[l])); }
          res_acc += res_w * cabs2(csub(yk, cscale(cadd(s1, cconj(s2)), a.inv_d)));
        }
      }
      // inverse split, scaled by 1/n (1/2 of the split times 1/N of the inverse)
#pragma unroll
      for (int l = 0; l < D2; ++l) {
        const float2 vbc = cconj(Vb[l]);
        const float2 E_ = cscale(cadd(Va[l], vbc), a.inv_n);
        const float2 O_ = cscale(cmulc(csub(Va[l], vbc), gw[k][l]), a.inv_n);
        lds[lpr(sa * LD + pa[l])] = cadd(E_, cmuli(O_));
        if (write_b) lds[lpr(sb * LD + qb[l])] = cconj(csub(E_, cmuli(O_)));
      }
    }
  } else {
    // Pointwise modes, by split pairs (k, N - k).  w > 0: slot 0 position p
    // pairs with slot 1 position N2-1-p.  w = 0: row 0 positions p in
    // [0, N2/2] pair with (N2 - p) mod N2 (p = 0 and N2/2 pair with
    // themselves), row N1/2 positions p < N2/2 pair with N2-1-p.
    const int np = (w0 ? N2 : (N2 + 1)) + (AI - 1) * N2;
    for (int gi = tid; gi < np; gi += T) {
      int pi, g;
      split_item(gi, N2, pi, g);
      const int w = w0 + pi;
      int sa, sb, rowa, p, mode;
      if (w) { sa = 2 * pi; sb = 2 * pi + 1; rowa = w; p = g; mode = 0; }
      else if (g <= (N2 >> 1)) { sa = 2 * pi; sb = 2 * pi; rowa = 0; p = g; mode = 1; }
      else { sa = 2 * pi + 1; sb = 2 * pi + 1; rowa = N1 >> 1; p = g - (N2 >> 1) - 1; mode = 2; }
      const int rowb = (mode == 0) ? (N1 - w) : rowa;
      const int q = (mode == 1) ? ((N2 - p) & (N2 - 1)) : (N2 - 1 - p);
      const bool write_b = !(mode == 1 && (p == 0 || p == (N2 >> 1)));
      const float2 za = lds[lpr(sa * LD + p)];
      const float2 zb = lds[lpr(sb * LD + q)];
      const float2 wt = cmul(a.twk1[rowa], a.twp[p]);
      const float2 zbc = cconj(zb);
      const float2 P = cscale(cadd(za, zbc), 0.5f);
      const float2 Q = cscale(cmulmi(csub(za, zbc)), 0.5f);
      const float2 wq = cmul(wt, Q);
      const float2 Xa = cadd(P, wq);
      const float2 Xb = cconj(csub(P, wq));
      if constexpr (OP == A_SPEC) {
        a.table[(size_t)rowa * N2 + p] = Xa;
        if (write_b) a.table[(size_t)rowb * N2 + q] = Xb;
        if (mode == 1 && p == 0) a.table[a.N] = Xb;
      } else if constexpr (SINGLE && OP != A_MUL && OP != A_MULC) {
        // d = 1: bins k (a) and N - k (b) are separate m-point bins, each
        // with its own y_hat.  Parseval weights over the n bins: bins 0 and
        // N once, a self-paired bin (N/2) twice on its own, every other bin
        // twice (itself and its conjugate).
        const bool edge = (mode == 1 && p == 0);
        const float2 ca = a.chat[(size_t)rowa * N2 + p];
        const float2 cb = edge ? a.chat[a.N] : a.chat[(size_t)rowb * N2 + q];
        const float2 ya = a.yhat[(size_t)rowa * N2 + p];
        const float2 yb = edge ? a.yhat[a.N] : a.yhat[(size_t)rowb * N2 + q];
        const float wa = edge ? 1.0f : 2.0f;
        const float wb = edge ? 1.0f : (write_b ? 2.0f : 0.0f);
        float2 Va, Vb;
        if constexpr (OP == A_RES) {
          res_acc += wa * cabs2(csub(ya, cmul(ca, Xa))) + wb * cabs2(csub(yb, cmul(cb, Xb)));
          continue;
        } else if constexpr (OP == A_ISTA) {
          // gradient step tau conj(c) (y_hat - c X); the column pass adds x
          const float2 ra = csub(ya, cmul(ca, Xa)), rb = csub(yb, cmul(cb, Xb));
          res_acc += wa * cabs2(ra) + wb * cabs2(rb);
          Va = cconjmul(ca, cscale(ra, tau));
          Vb = cconjmul(cb, cscale(rb, tau));
        } else {
          // Woodbury x-update in residual form with a single bin per class:
          // X' = W + conj(c) (y_hat - c W) / (rho + |c|^2)
          const float2 Ea = cscale(csub(ya, cmul(ca, Xa)), 1.0f / (a.rho + cabs2(ca)));
          const float2 Eb = cscale(csub(yb, cmul(cb, Xb)), 1.0f / (a.rho + cabs2(cb)));
          Va = cadd(Xa, cconjmul(ca, Ea));
          Vb = cadd(Xb, cconjmul(cb, Eb));
          if (a.res) res_acc += wa * cabs2(csub(ya, cmul(ca, Va))) + wb * cabs2(csub(yb, cmul(cb, Vb)));
        }
        const float2 vbc = cconj(Vb);
        const float2 E_ = cscale(cadd(Va, vbc), a.inv_n);
        const float2 O_ = cscale(cmulc(csub(Va, vbc), wt), a.inv_n);
        lds[lpr(sa * LD + p)] = cadd(E_, cmuli(O_));
        if (write_b) lds[lpr(sb * LD + q)] = cconj(csub(E_, cmuli(O_)));
      } else {
        const float2 ca = a.chat[(size_t)rowa * N2 + p];
        const float2 cb = (mode == 1 && p == 0) ? a.chat[a.N] : a.chat[(size_t)rowb * N2 + q];
        float2 Va, Vb;
        if constexpr (OP == A_MUL) { Va = cmul(ca, Xa); Vb = cmul(cb, Xb); }
        else { Va = cconjmul(ca, Xa); Vb = cconjmul(cb, Xb); }
        const float2 vbc = cconj(Vb);
        const float2 E_ = cscale(cadd(Va, vbc), a.inv_n);
        const float2 O_ = cscale(cmulc(csub(Va, vbc), wt), a.inv_n);
        lds[lpr(sa * LD + p)] = cadd(E_, cmuli(O_));
        if (write_b) lds[lpr(sb * LD + q)] = cconj(csub(E_, cmuli(O_)));
      }
    }
  }
  if constexpr (HAS_RES) {
    if (a.res) {
      const double r = block_sum<T>(double(res_acc), tid);
      if (tid == 0) a.res[w0] = r;   // (traces run with AI = 1)
    }
  }
  if constexpr (OP != A_SPEC && OP != A_RES) {
    __syncthreads();
    lds_fft<N2, 2 * AI, T, true, false, LD>(lds, tws, tid);
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
      const int i = tid + k * T;
      if (NR % T == 0 || i < NR) {
        const int s = i / N2, p = i % N2;
        Yg.st((size_t)row_of(s) * N2 + p, lds[lpr(s * LD + p)]);
      }
    }
  }
}

// Row-pass kernel: workgroup w owns rows {w, N1 - w}; workgroup 0 owns the
// two rows that are their own mirror images, {0, N1/2}.  The row-FFT stage
// twiddles W_{N2}^e are copied to LDS when both rows and the table fit in the
// 160 KiB of a CU, and read from the global table otherwise.
template <int N2, int OP, int D2>
__global__ __launch_bounds__(pass_a_threads(N2)) void k_passA(PassAArgs a) {
  constexpr int TA = pass_a_threads(N2);
  constexpr int LD = N2 + kPadA;
  constexpr bool TW_LDS = (lds_rows(2 * LD) + N2) * 8 <= 160 * 1024 - 1024;
  __shared__ float2 lds[lds_rows(2 * LD)];
  __shared__ float2 tws_l[TW_LDS ? N2 : 1];
  if constexpr (TW_LDS) {
    for (unsigned i = threadIdx.x; i < N2; i += TA) tws_l[i] = a.tw2[i];
  }
  __syncthreads();
  // long rows: class operands loaded after the forward transforms (three or
  // more classes per thread would otherwise be held across them)
  constexpr bool LATE = (N2 / (D2 > 0 ? D2 : 1) + 1 + TA - 1) / TA >= 3;
  rowpass<N2, OP, D2, TA, false, 1, LATE>(a, blockIdx.x, lds, TW_LDS ? tws_l : a.tw2, threadIdx.x);
}

// ---------------------------------------------------------------------------
// Pass B.  Workgroup b owns columns j2 in [b*CB, b*CB + CB); LDS holds them
// interleaved, element (column c, index i) at [i*CB + c].  Global accesses are
// issued in register-staged chunks of CH elements per thread so that a chunk's
// loads are all in flight before the first wait.
// Adjoint mask of one pair of samples: vbar = M_t * xbar with
// M_t = 1[|v_t| > theta_t]; accumulates -sgn(v_t) vbar_t (the threshold's
// derivative) and vbar_t * step_t (the step's, step_t = tau_t g_t) in double.
__device__ __forceinline__ float2 adj_mask(float2 xb, float2 v, float2 st, float thr, double& s_th, double& s_g) {
  const float2 vb = c2(fabsf(v.x) > thr ? xb.x : 0.0f, fabsf(v.y) > thr ? xb.y : 0.0f);
  s_th -= double(v.x > 0.0f ? vb.x : -vb.x) + double(v.y > 0.0f ? vb.y : -vb.y);
  s_g += double(vb.x) * double(st.x) + double(vb.y) * double(st.y);
  return vb;
}

// Workgroup sums of the two adjoint partials (wave shuffles, then one value
// per wave), written to part[0] and part[part_q].  All threads call it.
template <int T>
__device__ __forceinline__ void adj_partials(const PassBArgs& a, double s_th, double s_g, unsigned tid) {
  __shared__ double red[2][T / 64];
  for (int off = 32; off > 0; off >>= 1) {
    s_th += __shfl_xor(s_th, off);
    s_g += __shfl_xor(s_g, off);
  }
  if ((tid & 63) == 0) { red[0][tid >> 6] = s_th; red[1][tid >> 6] = s_g; }
  __syncthreads();
  if (tid == 0) {
    double r0 = 0.0, r1 = 0.0;
    for (int w = 0; w < T / 64; ++w) { r0 += red[0][w]; r1 += red[1][w]; }
    a.part[0] = r0;
    a.part[a.part_q] = r1;
  }
  __syncthreads();
}

// COH (persistent launches): device-coherent spectrum and state accesses, and
// (up to 8 values per thread) the state of B_ISTA / B_ADMM loaded together
// with the spectrum instead of after the inverse transform.  TWL:
// the four-step twiddles come from an LDS copy twn = [W_N^e, e < 2^lo_bits |
// W_N^(e 2^lo_bits), e < N >> lo_bits] instead of the global tables.
template <int N1, int MODE, int T, bool COH = false, int CBW = kColsPerBlock, bool TWL = false>
__device__ __forceinline__ void colpass(const PassBArgs& a, int blk, float2* __restrict__ lds,
                                        const float2* __restrict__ tws, unsigned tid,
                                        const float2* __restrict__ twn = nullptr) {
  constexpr int CB = CBW;   // adjacent columns held, interleaved
  constexpr int NE = N1 * CB;
  constexpr int EPT = (NE + T - 1) / T;
  constexpr int CH = EPT < 8 ? EPT : 8;
  constexpr bool FULL = (NE % T) == 0;
  const int j2_0 = blk * CB;
  const int N2 = a.N2;
  const Gf2<COH> Yg(a.Y, (unsigned)a.N);
  constexpr bool HAS_INV = (MODE == B_ISTA || MODE == B_ADMM || MODE == B_OUT_ALL || MODE == B_OUT_DEC ||
                            MODE == B_ISTA_REC || MODE == B_ADJ_X || MODE == B_ADJ_XV);
  constexpr bool STATE = (MODE == B_ISTA || MODE == B_ADMM || MODE == B_ISTA_REC);
  constexpr bool PRE = COH && STATE && EPT <= 8;   // state loaded with the spectrum (when it fits)
  auto twN = [&](int e) -> float2 {
    if constexpr (TWL) {
      e &= (a.N - 1);
      return cmul(twn[e & ((1 << a.lo_bits) - 1)], twn[(1 << a.lo_bits) + (e >> a.lo_bits)]);
    } else {
      return tw_N(a, e);
    }
  };
  const Gf2<COH> Sg(reinterpret_cast<float2*>(a.u), (unsigned)a.N);
  float2 svp[PRE ? EPT : 1];

  if constexpr (HAS_INV) {
#pragma unroll
    for (int k0 = 0; k0 < EPT; k0 += CH) {
      float2 v[CH], t[TWL ? 1 : CH];
#pragma unroll
      for (int k = 0; k < CH; ++k) {
        const int i = tid + (k0 + k) * T;
        if (FULL || i < NE) {
          const int k1 = i / CB, c = i % CB;
          const int j2 = j2_0 + c;
          v[k] = Yg.ld((size_t)k1 * N2 + j2);
          if constexpr (PRE) svp[k0 + k] = Sg.ld((size_t)k1 * N2 + j2);
          if constexpr (!TWL) t[k] = twN(j2 * k1);
        }
      }
#pragma unroll
      for (int k = 0; k < CH; ++k) {
        const int i = tid + (k0 + k) * T;
        if (FULL || i < NE) {
          if constexpr (TWL) lds[lp(i)] = cmulc(v[k], twN((j2_0 + (i % CB)) * (i / CB)));
          else lds[lp(i)] = cmulc(v[k], t[k]);
        }
      }
    }
    __syncthreads();
    lds_fft<N1, CB, T, true, true, N1>(lds, tws, tid);
    // time domain: lds[lp(j1*CB + c)] = (x_{2j}, x_{2j+1}), j = N2*j1 + j2_0 + c
    bool fwd = true;
    if constexpr (MODE == B_ISTA || MODE == B_ADMM || MODE == B_ISTA_REC) {
      // ISTA: lds holds tau A^T r and a.u is the iterate x.
      // ADMM: lds holds x(t) and a.u is the scaled dual u.
      const float thr = a.tau_dev ? a.tau_dev[a.t] * a.lam_dev[a.t] : a.thr;
      float l1_acc = 0.0f;   // objective trace: sum |x| of this thread's samples
#pragma unroll
      for (int k0 = 0; k0 < EPT; k0 += CH) {
        float2 sv[CH];
#pragma unroll
        for (int k = 0; k < CH; ++k) {
          const int i = tid + (k0 + k) * T;
          if constexpr (PRE) sv[k] = svp[k0 + k];
          else if (FULL || i < NE) sv[k] = Sg.ld((size_t)(i / CB) * N2 + j2_0 + (i % CB));
        }
#pragma unroll
        for (int k = 0; k < CH; ++k) {
          const int i = tid + (k0 + k) * T;
          if (FULL || i < NE) {
            const size_t j = (size_t)(i / CB) * N2 + j2_0 + (i % CB);
            if constexpr (MODE == B_ISTA || MODE == B_ISTA_REC) {
              const float2 step = lds[lp(i)];
              const float2 v = cadd(sv[k], step);
              const float2 x = c2(soft(v.x, thr), soft(v.y, thr));
              l1_acc += fabsf(x.x) + fabsf(x.y);
              Sg.st(j, x);
              lds[lp(i)] = x;
              if constexpr (MODE == B_ISTA_REC) {
                reinterpret_cast<float2*>(a.rv)[j] = v;
                reinterpret_cast<float2*>(a.rd)[j] = step;
              }
            } else {
              const float2 x = lds[lp(i)];
              l1_acc += fabsf(x.x) + fabsf(x.y);
              const float2 xu = cadd(x, sv[k]);
              const float2 z = c2(soft(xu.x, thr), soft(xu.y, thr));
              const float2 u1 = csub(xu, z);
              Sg.st(j, u1);
              if (a.last) {
                reinterpret_cast<float2*>(a.out0)[j] = x;
                reinterpret_cast<float2*>(a.out1)[j] = z;
              } else {
                lds[lp(i)] = csub(z, u1);
              }
            }
          }
        }
      }
      if (a.l1) {
        const double r = block_sum<T>(double(l1_acc), tid);
        if (tid == 0) a.l1[blk] = r;
      }
      fwd = !a.last;
    } else if constexpr (MODE == B_ADJ_X) {
      // xbar_{t-1} = vbar_t - tau_t A^T A vbar_t (lds holds the second term)
      for (int i = tid; i < NE; i += T) {
        const size_t j = (size_t)(i / CB) * N2 + j2_0 + (i % CB);
        reinterpret_cast<float2*>(a.xbar)[j] = cadd(reinterpret_cast<const float2*>(a.vbar)[j], lds[lp(i)]);
      }
      fwd = false;
    } else if constexpr (MODE == B_ADJ_XV) {
      // xbar_{t-1} = vbar_t + lds, then step t-1's mask and sums in place
      const float thr = a.tau_dev[a.t] * a.lam_dev[a.t];
      double s_th = 0.0, s_g = 0.0;
      for (int i = tid; i < NE; i += T) {
        const size_t j = (size_t)(i / CB) * N2 + j2_0 + (i % CB);
        const float2 xb = cadd(reinterpret_cast<const float2*>(a.vbar)[j], lds[lp(i)]);
        const float2 vb = adj_mask(xb, reinterpret_cast<const float2*>(a.rv)[j],
                                   reinterpret_cast<const float2*>(a.rd)[j], thr, s_th, s_g);
        reinterpret_cast<float2*>(a.vbar)[j] = vb;
        lds[lp(i)] = vb;
      }
      adj_partials<T>(a, s_th, s_g, tid);
    } else if constexpr (MODE == B_OUT_ALL) {
      for (int i = tid; i < NE; i += T) {
        const int j1 = i / CB, c = i % CB;
        const size_t j = (size_t)j1 * N2 + j2_0 + c;
        reinterpret_cast<float2*>(a.out0)[j] = lds[lp(i)];
      }
      fwd = false;
    } else {  // B_OUT_DEC: real sample 2j is kept when 2j % d == 0 (d even; d = 1 keeps all)
      const int h = a.d >> 1;
      for (int i = tid; i < NE; i += T) {
        const int j1 = i / CB, c = i % CB;
        const size_t j = (size_t)j1 * N2 + j2_0 + c;
        if (h == 0) reinterpret_cast<float2*>(a.out0)[j] = lds[lp(i)];
        else if ((j % h) == 0) a.out0[j / h] = lds[lp(i)].x;
      }
      fwd = false;
    }
    if (!fwd) return;
    __syncthreads();
  } else if constexpr (MODE == B_ADJ_V) {
    // vbar_t = M_t * xbar_t with M_t = 1[|v_t| > theta_t]; per-workgroup sums
    // of -sgn(v_t) vbar_t (threshold derivative) and vbar_t * step_t (the
    // step's derivative, step_t = tau_t g_t), accumulated in double
    const float thr = a.tau_dev[a.t] * a.lam_dev[a.t];
    double s_th = 0.0, s_g = 0.0;
    for (int i = tid; i < NE; i += T) {
      const size_t j = (size_t)(i / CB) * N2 + j2_0 + (i % CB);
      const float2 vb = adj_mask(reinterpret_cast<const float2*>(a.xbar)[j], reinterpret_cast<const float2*>(a.rv)[j],
                                 reinterpret_cast<const float2*>(a.rd)[j], thr, s_th, s_g);
      reinterpret_cast<float2*>(a.vbar)[j] = vb;
      lds[lp(i)] = vb;
    }
    adj_partials<T>(a, s_th, s_g, tid);
  } else {
#pragma unroll
    for (int k0 = 0; k0 < EPT; k0 += CH) {
      float2 v[CH];
#pragma unroll
      for (int k = 0; k < CH; ++k) {
        const int i = tid + (k0 + k) * T;
        if (FULL || i < NE) {
          const size_t j = (size_t)(i / CB) * N2 + j2_0 + (i % CB);
          if constexpr (MODE == B_FWD_REAL) {
            v[k] = reinterpret_cast<const float2*>(a.in0)[j];
          } else if constexpr (MODE == B_FWD_UP) {
            // P^T r: r_i at real sample d i; pair j holds samples 2j, 2j + 1
            const int h = a.d >> 1;
            if (h == 0) v[k] = reinterpret_cast<const float2*>(a.in0)[j];
            else v[k] = c2((j % h) == 0 ? a.in0[j / h] : 0.0f, 0.0f);
          } else {
            v[k] = csub(reinterpret_cast<const float2*>(a.in0)[j], reinterpret_cast<const float2*>(a.in1)[j]);
          }
        }
      }
#pragma unroll
      for (int k = 0; k < CH; ++k) {
        const int i = tid + (k0 + k) * T;
        if (FULL || i < NE) lds[lp(i)] = v[k];
      }
    }
    __syncthreads();
  }
  lds_fft<N1, CB, T, false, true, N1>(lds, tws, tid);
#pragma unroll
  for (int k0 = 0; k0 < EPT; k0 += CH) {
    float2 t[CH];
#pragma unroll
    for (int k = 0; k < CH; ++k) {
      const int i = tid + (k0 + k) * T;
      if (FULL || i < NE) t[k] = twN((j2_0 + (i % CB)) * (i / CB));
    }
#pragma unroll
    for (int k = 0; k < CH; ++k) {
      const int i = tid + (k0 + k) * T;
      if (FULL || i < NE) {
        const int k1 = i / CB, c = i % CB;
        Yg.st((size_t)k1 * N2 + j2_0 + c, cmul(lds[lp(i)], t[k]));
      }
    }
  }
}


// Columns per column-pass workgroup of the two-launch schedule: 8 (64-byte
// runs); 4 for 4096-point columns, whose 8-column block would not fit LDS.
constexpr int pass_b_cols(int N1) { return N1 > 2048 ? 4 : kColsPerBlock; }

#ifndef CS_PASSB_XCD
#define CS_PASSB_XCD 1
#endif

// Column block of the column pass's workgroup b.  Workgroups are dispatched
// round-robin over the 8 XCDs, each with its own L2; a column block's rows are
// CB * 8 bytes, less than a 128-byte line, so neighbouring blocks share lines.
// XCD x takes the contiguous range [x G/8, (x + 1) G/8) in order, so the
// workgroups resident on one XCD at a time read and write whole lines through
// the same L2 (a permutation of the blocks whenever G is a multiple of 8).
__device__ __forceinline__ int passb_block(unsigned b, unsigned G) {
  if (CS_PASSB_XCD && (G & 7u) == 0) return (int)((b & 7u) * (G >> 3) + (b >> 3));
  return (int)b;
}

// Column-pass kernel: the workgroup owns columns [CB blk, CB blk + CB), blk
// as above.  The stage twiddles are staged in LDS up to 2048-point columns
// and read from the global table above.
template <int N1, int MODE>
__global__ __launch_bounds__(pass_b_threads(N1)) void k_passB(PassBArgs a) {
  constexpr int TB = pass_b_threads(N1);
  constexpr int CB = pass_b_cols(N1);
  constexpr bool TWL = N1 <= 2048;
  __shared__ float2 lds[lds_padded(N1 * CB)];
  __shared__ float2 tws_l[TWL ? N1 : 1];
  if constexpr (TWL)
    for (unsigned i = threadIdx.x; i < N1; i += TB) tws_l[i] = a.tw1[i];
  __syncthreads();
  colpass<N1, MODE, TB, false, CB>(a, passb_block(blockIdx.x, gridDim.x), lds, TWL ? tws_l : a.tw1, threadIdx.x);
}

}  // namespace cs
