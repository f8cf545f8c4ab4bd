// Direct (FFT-free) products with the partial circulant A = P C: every output
// is an inner product over the generator c, as in the paper's GPU kernels
// (Section 4: the CPISTA residual kernel forms a row of A times x, the
// thresholded-gradient kernel a row of A^T times r, reading only c and never
// forming A).  O(n m) multiply-adds per product, against O(n log n) for the
// FFT path: a baseline that measures what the FFT formulation buys on this
// GPU, not a solver path.
//
//   y_i = sum_{j < n} c[(d i - j) mod n] x_j,   i < m = n/d      (A x)
//   x_j = sum_{i < m} c[(d i - j) mod n] r_i,   j < n            (A^T r)
//
// A workgroup owns a tile of outputs and walks the inputs in tiles.  For an
// output tile and an input tile the c values involved form one contiguous
// window of c (indices d i - j over the two tiles), staged in LDS with the
// input tile; each thread then accumulates its outputs in registers.
// Forward: thread t owns outputs i0 + t + q*T (q < RO), so for a block of four
// inputs the four c values of one output are contiguous (one 16-byte LDS
// read per four multiply-adds, consecutive lanes 4d bytes apart) and the four
// inputs are a broadcast read.  Transpose: a register sliding window along
// the d-strided diagonals (one 4-byte LDS read per RO multiply-adds, see
// k_direct_adj) with r_i a broadcast.
// Accumulation is in FP32, in input order.  The next tile's window and inputs
// are loaded into registers while the current tile is computed, so the
// global loads of the staging overlap the multiply-adds.
#pragma once
#include <hip/hip_runtime.h>

namespace cs {

constexpr int kDirT = 256;          // threads per workgroup
constexpr int kDirTileJ = 1024;     // forward: inputs per tile (min(n, 1024))
constexpr int kDirTileI = 512;      // transpose: inputs per tile (min(m, 512))
constexpr int kDirOutT = 2048;      // transpose: outputs per workgroup

template <int D>
constexpr int dir_fwd_outputs() { return 8192 / D; }   // forward outputs per workgroup

// y = A x.  Grid: ceil(m / dir_fwd_outputs<D>()) workgroups of kDirT threads.
template <int D>
__global__ __launch_bounds__(kDirT) void k_direct_fwd(const float* __restrict__ c, const float* __restrict__ x,
                                                      float* __restrict__ y, long long n) {
  constexpr int TI = dir_fwd_outputs<D>();
  constexpr int RO = TI / kDirT;
  __shared__ __align__(16) float xs[kDirTileJ];
  __shared__ __align__(16) float cw[D * TI + kDirTileJ];
  const long long m = n / D;
  const long long i0 = (long long)blockIdx.x * TI;
  const int tid = threadIdx.x;
  const int tile = n < kDirTileJ ? (int)n : kDirTileJ;
  const long long mask = n - 1;
  float acc[RO];
#pragma unroll
  for (int q = 0; q < RO; ++q) acc[q] = 0.0f;
  // window of tile j0: cw[u] = c[(D i0 - j0 - tile + 1 + u) mod n], u < D TI + tile
  constexpr int NW = (D * TI + kDirTileJ) / kDirT;   // window values per thread
  constexpr int NX = kDirTileJ / kDirT;              // inputs per thread
  float pw[NW], px[NX];
  auto fetch = [&](long long j0) {
    const long long base = (D * i0 - j0 - tile + 1) & mask;
#pragma unroll
    for (int k = 0; k < NW; ++k) {
      const int u = tid + k * kDirT;
      if (u < D * TI + tile) pw[k] = c[(base + u) & mask];
    }
#pragma unroll
    for (int k = 0; k < NX; ++k) {
      const int u = tid + k * kDirT;
      if (u < tile) px[k] = x[j0 + u];
    }
  };
  fetch(0);
  for (long long j0 = 0; j0 < n; j0 += tile) {
#pragma unroll
    for (int k = 0; k < NW; ++k) {
      const int u = tid + k * kDirT;
      if (u < D * TI + tile) cw[u] = pw[k];
    }
#pragma unroll
    for (int k = 0; k < NX; ++k) {
      const int u = tid + k * kDirT;
      if (u < tile) xs[u] = px[k];
    }
    __syncthreads();
    if (j0 + tile < n) fetch(j0 + tile);
    // output i = i0 + tid + q T, input j = j0 + jj:  u = D (tid + q T) - jj + tile - 1;
    // the four c values for jj = jb + 3 .. jb start at s0 = D (tid + q T) +
    // tile - 4 - jb, a multiple of 4 (of 2 for D = 2), read through a vector
    // index so the 16-byte (8-byte) alignment is explicit: element-wise
    // addressing lets the compiler split the read into 4-byte pairs, which
    // conflict on the banks at this lane stride
    const float4* xs4 = reinterpret_cast<const float4*>(xs);
    const float4* cw4 = reinterpret_cast<const float4*>(cw);
    const float2* cw2 = reinterpret_cast<const float2*>(cw);
    for (int jb = 0; jb < tile; jb += 4) {
      const float4 xv = xs4[jb >> 2];
#pragma unroll
      for (int q = 0; q < RO; ++q) {
        float4 cv;
        if constexpr (D % 4 == 0) {
          cv = cw4[(D / 4) * (tid + q * kDirT) + ((tile - jb) >> 2) - 1];
        } else {
          const int h0 = (D / 2) * (tid + q * kDirT) + ((tile - 4 - jb) >> 1);
          const float2 lo = cw2[h0];
          const float2 hi = cw2[h0 + 1];
          cv = make_float4(lo.x, lo.y, hi.x, hi.y);
        }
        acc[q] = fmaf(cv.w, xv.x, acc[q]);
        acc[q] = fmaf(cv.z, xv.y, acc[q]);
        acc[q] = fmaf(cv.y, xv.z, acc[q]);
        acc[q] = fmaf(cv.x, xv.w, acc[q]);
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < RO; ++q) {
    const long long i = i0 + tid + (long long)q * kDirT;
    if (i < m) y[i] = acc[q];
  }
}

// x = A^T r.  Grid: ceil(n / kDirOutT) workgroups of kDirT threads.
//
// Thread t = a + D b (a < D) owns outputs j0 + a + D (b RO + q), q < RO.  For
// input i0 + ii its c index is u = D (ii - b RO - q) - a + kDirOutT - 1: all of
// a thread's indices share the residue D - 1 - a of u mod D, and along
// w = ii - q they are consecutive in u / D, so the values of one thread form a
// sliding window: each new input brings one new value and the other RO - 1
// are reused from registers (one LDS read per RO multiply-adds).  The c
// window is stored split by residue class, each class padded with one word
// per 2^SH and offset by a per-d extra stride, which makes the reads of the
// 64 lanes of a wave hit 64 distinct banks for every d (checked on the host
// with a bank model).
template <int D>
struct DirAdjLayout {
  static constexpr int SH = (D == 2) ? 2 : 3;
  static constexpr int XS = (D == 2) ? 1 : (D == 4) ? 8 : (D == 8) ? 0 : 4;
  static constexpr int LV = kDirOutT / D + kDirTileI;          // u / D range of the window
  static constexpr int LVP = LV + (LV >> SH) + 8 + XS;         // padded length of one class
  __device__ static int pv(int v) { return v + (v >> SH); }
};

template <int D>
__global__ __launch_bounds__(kDirT) void k_direct_adj(const float* __restrict__ c, const float* __restrict__ r,
                                                      float* __restrict__ x, long long n) {
  using Lay = DirAdjLayout<D>;
  constexpr int RO = kDirOutT / kDirT;
  __shared__ float rs[kDirTileI];
  __shared__ float cw[D * Lay::LVP];
  const long long m = n / D;
  const long long j0 = (long long)blockIdx.x * kDirOutT;
  const int tid = threadIdx.x;
  const int tile = m < kDirTileI ? (int)m : kDirTileI;
  const long long mask = n - 1;
  const int a = tid % D, b = tid / D;
  const float* cr = cw + (D - 1 - a) * Lay::LVP;
  const int vb = kDirOutT / D - 1 - b * RO;   // u / D of (ii, q) is vb + ii - q
  float acc[RO];
#pragma unroll
  for (int q = 0; q < RO; ++q) acc[q] = 0.0f;
  // window of tile i0: c[(D i0 - j0 - kDirOutT + 1 + u) mod n] for
  // u < D tile + kDirOutT, stored at cw[(u mod D) LVP + pv(u / D)]
  constexpr int NW = (D * kDirTileI + kDirOutT) / kDirT;
  constexpr int NR = kDirTileI / kDirT;
  float pw[NW], pr[NR];
  auto fetch = [&](long long i0) {
    const long long base = (D * i0 - j0 - kDirOutT + 1) & mask;
#pragma unroll
    for (int k = 0; k < NW; ++k) {
      const int u = tid + k * kDirT;
      if (u < D * tile + kDirOutT) pw[k] = c[(base + u) & mask];
    }
#pragma unroll
    for (int k = 0; k < NR; ++k) {
      const int u = tid + k * kDirT;
      if (u < tile) pr[k] = r[i0 + u];
    }
  };
  fetch(0);
  for (long long i0 = 0; i0 < m; i0 += tile) {
#pragma unroll
    for (int k = 0; k < NW; ++k) {
      const int u = tid + k * kDirT;
      if (u < D * tile + kDirOutT) cw[(u % D) * Lay::LVP + Lay::pv(u / D)] = pw[k];
    }
#pragma unroll
    for (int k = 0; k < NR; ++k) {
      const int u = tid + k * kDirT;
      if (u < tile) rs[u] = pr[k];
    }
    __syncthreads();
    if (i0 + tile < m) fetch(i0 + tile);
    // prev[RO + w] holds the value at w = ii - q < 0 of the current chunk
    float prev[RO];
#pragma unroll
    for (int w = 1; w < RO; ++w) prev[RO - w] = cr[Lay::pv(vb - w)];
    for (int ii0 = 0; ii0 < tile; ii0 += RO) {
      float cur[RO];
#pragma unroll
      for (int s = 0; s < RO; ++s) cur[s] = cr[Lay::pv(vb + ii0 + s)];
#pragma unroll
      for (int s = 0; s < RO; ++s) {
        const float rv = rs[ii0 + s];
#pragma unroll
        for (int q = 0; q < RO; ++q) acc[q] = fmaf(s >= q ? cur[s - q] : prev[RO + s - q], rv, acc[q]);
      }
#pragma unroll
      for (int s = 1; s < RO; ++s) prev[s] = cur[s];
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < RO; ++q) {
    const long long j = j0 + a + (long long)D * (b * RO + q);
    if (j < n) x[j] = acc[q];
  }
}

}  // namespace cs
