// Workgroup-wide complex FFTs held in LDS: Stockham autosort with radix-16
// stages and one radix-2/4/8 stage for the remaining factor.
//
// Algorithm: the self-sorting Stockham formulation (C. Van Loan, Computational
// Frameworks for the Fast Fourier Transform, SIAM 1992, Section 1.7).  Stage s
// with span Ns (product of the radices already applied) and radix R reads, for
// butterfly j < L/R, the R elements j + r*L/R, multiplies element r by
// W_{Ns*R}^{r*(j mod Ns)}, takes an R-point DFT and writes element r to
// (j - j mod Ns)*R + (j mod Ns) + r*Ns.  The output is in natural order.
//
// Data layout: B independent sequences of length L.
//   ILV = false: sequence b, element i at buf[b*LD + i]        (rows)
//   ILV = true : sequence b, element i at buf[i*B + b]         (interleaved
//                columns; consecutive threads take consecutive b so every
//                LDS access of a stage is unit-stride across the wave)
// Each stage loads its butterflies into registers, barriers, then stores in
// place, so LDS holds one copy of the data.  Every LDS address goes through
// lp() below.  Twiddles come from a table tw[e] = exp(-2 pi i e / L), e < L,
// computed on the host in double precision; a butterfly reads at most three
// of them and forms its other powers by complex products.
// Forward transforms use exp(-...), inverse ones exp(+...), both unnormalised.
#pragma once
#include "cplx.hpp"

namespace cs {

constexpr int ilog2c(int v) { return v <= 1 ? 0 : 1 + ilog2c(v / 2); }

#ifndef CS_MAX_RADIX
#define CS_MAX_RADIX 8
#endif

// Radix of the stage that starts at span NS.
// Radix-16 plan: 16 while at least 16 remains; a leftover factor of 2 is
// avoided by ending with 8 * 4.  Radix-8 plan: radix 8, with one radix-4 (or
// radix-2) stage first where log2(L) is not a multiple of three.
constexpr int stage_radix(int L, int NS) {
  const int p = ilog2c(L / NS);
  if (CS_MAX_RADIX >= 16) {
    if (p >= 4 && p != 5) return 16;
    if (p == 5) return 8;
    return 1 << p;
  }
  return (p % 3 == 0) ? 8 : ((p % 3 == 2) ? 4 : (p == 1 ? 2 : 4));
}

// LDS slot of flat index x in interleaved (column) buffers: identity.
// Bank swizzles and per-32 padding applied through a per-access function
// were measured slower on gfx950: they stop the compiler from folding
// constant offsets into paired ds_read2 / ds_write2 accesses.
__device__ __forceinline__ unsigned lp(unsigned x) { return x; }
constexpr int lds_padded(int n) { return n; }

#ifndef CS_ROW_PAD
#define CS_ROW_PAD 1
#endif
// Row buffers (sequences stored one after another): with CS_ROW_PAD one pad
// slot follows every 32 slots, which moves the strided stores of the early
// Stockham stages off the banks they would otherwise share.  The FFT stages
// compute one padded base per butterfly and add compile-time offsets (valid
// for power-of-two radices, spans and row lengths that are multiples of 32).
__device__ __forceinline__ unsigned lpr(unsigned x) { return CS_ROW_PAD ? x + (x >> 5) : x; }
constexpr int lds_rows(int n) { return CS_ROW_PAD ? n + n / 32 + 1 : n; }
constexpr unsigned prc(unsigned x) { return CS_ROW_PAD ? x + x / 32 : x; }

// multiply by the primitive 8th root of unity W8^q (q = 1, 3), forward sign
// exp(-i pi q / 4) or inverse sign exp(+i pi q / 4).
template <bool INV>
__device__ __forceinline__ float2 mul_w8_1(float2 a) {
  const float s = 0.70710678118654752440f;
  // fwd: (1 - i)/sqrt2 * (x + iy) = ((x + y) + i(y - x))/sqrt2
  // inv: (1 + i)/sqrt2 * (x + iy) = ((x - y) + i(x + y))/sqrt2
  return INV ? c2((a.x - a.y) * s, (a.x + a.y) * s) : c2((a.x + a.y) * s, (a.y - a.x) * s);
}
template <bool INV>
__device__ __forceinline__ float2 mul_w8_3(float2 a) {
  const float s = 0.70710678118654752440f;
  // fwd: (-1 - i)/sqrt2 * (x + iy) = ((y - x) - i(x + y))/sqrt2
  // inv: (-1 + i)/sqrt2 * (x + iy) = (-(x + y) + i(x - y))/sqrt2
  return INV ? c2(-(a.x + a.y) * s, (a.x - a.y) * s) : c2((a.y - a.x) * s, -(a.x + a.y) * s);
}
template <bool INV>
__device__ __forceinline__ float2 mul_w4(float2 a) {  // W4 = -i (fwd), +i (inv)
  return INV ? cmuli(a) : cmulmi(a);
}

template <bool INV>
__device__ __forceinline__ void dft2(float2* v) {
  const float2 a = v[0];
  v[0] = cadd(a, v[1]);
  v[1] = csub(a, v[1]);
}

template <bool INV>
__device__ __forceinline__ void dft4(float2& v0, float2& v1, float2& v2, float2& v3) {
  const float2 a = cadd(v0, v2), b = csub(v0, v2);
  const float2 c = cadd(v1, v3), d = mul_w4<INV>(csub(v1, v3));
  v0 = cadd(a, c);
  v2 = csub(a, c);
  v1 = cadd(b, d);
  v3 = csub(b, d);
}

template <bool INV>
__device__ __forceinline__ void dft8(float2* v) {
  // even/odd split: E = DFT4(v0, v2, v4, v6), O = DFT4(v1, v3, v5, v7);
  // y_k = E_k + W8^k O_k, y_{k+4} = E_k - W8^k O_k.
  float2 e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
  float2 o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
  dft4<INV>(e0, e1, e2, e3);
  dft4<INV>(o0, o1, o2, o3);
  o1 = mul_w8_1<INV>(o1);
  o2 = mul_w4<INV>(o2);
  o3 = mul_w8_3<INV>(o3);
  v[0] = cadd(e0, o0); v[4] = csub(e0, o0);
  v[1] = cadd(e1, o1); v[5] = csub(e1, o1);
  v[2] = cadd(e2, o2); v[6] = csub(e2, o2);
  v[3] = cadd(e3, o3); v[7] = csub(e3, o3);
}

// 16-point DFT as 4 x 4: with r = 4a + b and k = c + 4d,
// W16^{rk} = W4^{ac} W16^{bc} W4^{bd}: DFT4 over a for each b, twiddle by
// W16^{bc}, DFT4 over b for each c.
template <bool INV>
__device__ __forceinline__ void dft16(float2* v) {
  const float c1 = 0.92387953251128675613f, s1 = 0.38268343236508977173f;  // cos, sin of pi/8
  // step 1: t[b][c] in place at v[4c + b]... computed per b over a
#pragma unroll
  for (int b = 0; b < 4; ++b) dft4<INV>(v[b], v[4 + b], v[8 + b], v[12 + b]);
  // now v[4c + b] = t[b][c]; step 2: twiddle W16^{bc} (conjugated for INV)
  auto tw = [&](float2 a, float cr, float ci) {   // a * (cr + i ci) with ci sign per direction
    const float si = INV ? -ci : ci;
    return c2(fmaf(a.x, cr, -a.y * si), fmaf(a.x, si, a.y * cr));
  };
  // W16^1 = (c1, -s1), W16^2 = W8^1, W16^3 = (s1, -c1), W16^4 = -i, W16^6 = W8^3, W16^9 = (-c1, s1)
  v[4 + 1] = tw(v[4 + 1], c1, -s1);          // b=1, c=1
  v[8 + 1] = mul_w8_1<INV>(v[8 + 1]);        // b=1, c=2
  v[12 + 1] = tw(v[12 + 1], s1, -c1);        // b=1, c=3
  v[4 + 2] = mul_w8_1<INV>(v[4 + 2]);        // b=2, c=1
  v[8 + 2] = mul_w4<INV>(v[8 + 2]);          // b=2, c=2
  v[12 + 2] = mul_w8_3<INV>(v[12 + 2]);      // b=2, c=3
  v[4 + 3] = tw(v[4 + 3], s1, -c1);          // b=3, c=1
  v[8 + 3] = mul_w8_3<INV>(v[8 + 3]);        // b=3, c=2
  v[12 + 3] = tw(v[12 + 3], -c1, s1);        // b=3, c=3
  // step 3: for each c, DFT4 over b: y[c + 4d] = sum_b t[b][c] W4^{bd}
  float2 y[16];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    float2 a0 = v[4 * c], a1 = v[4 * c + 1], a2 = v[4 * c + 2], a3 = v[4 * c + 3];
    dft4<INV>(a0, a1, a2, a3);
    y[c] = a0; y[c + 4] = a1; y[c + 8] = a2; y[c + 12] = a3;
  }
#pragma unroll
  for (int k = 0; k < 16; ++k) v[k] = y[k];
}

template <int R, bool INV>
__device__ __forceinline__ void dft(float2* v) {
  if constexpr (R == 2) dft2<INV>(v);
  else if constexpr (R == 4) dft4<INV>(v[0], v[1], v[2], v[3]);
  else if constexpr (R == 8) dft8<INV>(v);
  else dft16<INV>(v);
}

template <bool ILV, int B, int LD>
__device__ __forceinline__ unsigned lds_addr(unsigned b, unsigned i) {
  if constexpr (ILV) return lp(i * B + b);
  else return lpr(b * LD + i);
}

template <int L, int B, int T, bool INV, bool ILV, int LD, int NS, int R>
__device__ __forceinline__ void stockham_stage(float2* __restrict__ buf,
                                               const float2* __restrict__ tw, unsigned tid) {
  constexpr int Q = L / R;          // butterflies per sequence
  constexpr int NBF = B * Q;        // butterflies per stage
  constexpr int PER = (NBF + T - 1) / T;
  float2 v[PER][R];
  // explicit padded bases need rows that start on 32-slot blocks; otherwise
  // the per-access map lds_addr (the same mapping) is used
  constexpr bool PADR = CS_ROW_PAD && !ILV && (B == 1 || LD % 32 == 0);
  constexpr unsigned LDP = prc(LD);   // padded row stride
#pragma unroll
  for (int p = 0; p < PER; ++p) {
    const unsigned i = tid + p * T;
    if (NBF % T == 0 || i < NBF) {
      const unsigned b = ILV ? (i % B) : (i / Q);
      const unsigned j = ILV ? (i / B) : (i % Q);
      if constexpr (PADR) {
        const unsigned rb = b * LDP + lpr(j);
#pragma unroll
        for (int r = 0; r < R; ++r) v[p][r] = buf[rb + prc(r * Q)];
      } else {
#pragma unroll
        for (int r = 0; r < R; ++r) v[p][r] = buf[lds_addr<ILV, B, LD>(b, j + r * Q)];
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int p = 0; p < PER; ++p) {
    const unsigned i = tid + p * T;
    if (NBF % T == 0 || i < NBF) {
      const unsigned b = ILV ? (i % B) : (i / Q);
      const unsigned j = ILV ? (i / B) : (i % Q);
      const unsigned k = j & (NS - 1);
      if constexpr (NS > 1) {
        // twiddles W_{NS R}^{r k}: read W^k (and W^{4k}, W^{8k} for the
        // larger radices) from the table and form the other powers by
        // products (chains of at most three), so a butterfly makes at most
        // three LDS gathers instead of R - 1
        constexpr unsigned S = L / (NS * R);
        float2 w[R];
        w[1] = tw[k * S];
        if constexpr (R >= 4) {
          w[2] = cmul(w[1], w[1]);
          w[3] = cmul(w[2], w[1]);
        }
        if constexpr (R >= 8) {
          w[4] = tw[4 * k * S];
          w[5] = cmul(w[4], w[1]);
          w[6] = cmul(w[4], w[2]);
          w[7] = cmul(w[4], w[3]);
        }
        if constexpr (R >= 16) {
          w[8] = tw[8 * k * S];
#pragma unroll
          for (int r = 9; r < 16; ++r) w[r] = cmul(w[8], w[r - 8]);
        }
#pragma unroll
        for (int r = 1; r < R; ++r) v[p][r] = INV ? cmulc(v[p][r], w[r]) : cmul(v[p][r], w[r]);
      }
      dft<R, INV>(v[p]);
      const unsigned base = (j - k) * R + k;
      if constexpr (PADR) {
        const unsigned wb = b * LDP + lpr(base);
#pragma unroll
        for (int r = 0; r < R; ++r) buf[wb + prc(r * NS)] = v[p][r];
      } else {
#pragma unroll
        for (int r = 0; r < R; ++r) buf[lds_addr<ILV, B, LD>(b, base + r * NS)] = v[p][r];
      }
    }
  }
  __syncthreads();
}

// B transforms of length L (power of two, >= 2) in place in LDS; all T threads
// of the workgroup must call it.  Barriers are included before and after
// every stage's stores; the caller barriers before the first call.
template <int L, int B, int T, bool INV, bool ILV, int LD, int NS = 1>
__device__ __forceinline__ void lds_fft(float2* __restrict__ buf,
                                        const float2* __restrict__ tw, unsigned tid) {
  if constexpr (NS < L) {
    constexpr int R = stage_radix(L, NS);
    stockham_stage<L, B, T, INV, ILV, LD, NS, R>(buf, tw, tid);
    lds_fft<L, B, T, INV, ILV, LD, NS * R>(buf, tw, tid);
  }
}

// ---------------------------------------------------------------------------
// Transforms whose first and last stages run in registers.  A caller that
// already holds, for butterfly j < L/8 of sequence b, the eight elements
// j + r*L/8 (r < 8) takes the first radix-8 stage (span 1) with
// reg_stage_first, which leaves its outputs in LDS; lds_fft_mid runs the
// stages between spans 8 and L/8 through LDS; reg_stage_last loads the last
// radix-8 stage's inputs (span L/8, again the elements j + r*L/8 of each
// butterfly) and leaves its outputs in registers, in natural order at the
// same positions j + r*L/8.  This saves the LDS round trip at each end of
// the transform, so a load from global memory, a pointwise step between two
// transforms, or a store to global memory works on registers.  L >= 64.
// Callers barrier after reg_stage_first's stores and before anything
// overwrites the LDS that reg_stage_last reads.
template <int L, int B, bool INV, bool ILV, int LD>
__device__ __forceinline__ void reg_stage_first(float2* __restrict__ buf, float2 (&v)[8], unsigned b,
                                                unsigned j) {
  static_assert(L >= 64, "");
  dft8<INV>(v);
  // positions j*8 + r: one base plus constant offsets (r < 8 never crosses
  // a 32-slot pad block because j*8 is a multiple of 8)
  constexpr bool PADR = CS_ROW_PAD && !ILV && (B == 1 || LD % 32 == 0);
  if constexpr (ILV) {
    const unsigned base = (j * 8) * B + b;
#pragma unroll
    for (int r = 0; r < 8; ++r) buf[lp(base + r * B)] = v[r];
  } else if constexpr (PADR) {
    const unsigned base = b * prc(LD) + lpr(j * 8);
#pragma unroll
    for (int r = 0; r < 8; ++r) buf[base + r] = v[r];
  } else {
#pragma unroll
    for (int r = 0; r < 8; ++r) buf[lds_addr<ILV, B, LD>(b, j * 8 + r)] = v[r];
  }
}

template <int L, int B, bool INV, bool ILV, int LD>
__device__ __forceinline__ void reg_stage_last(const float2* __restrict__ buf, const float2* __restrict__ tw,
                                               float2 (&v)[8], unsigned b, unsigned j) {
  static_assert(L >= 64, "");
  constexpr unsigned Q = L / 8;
  constexpr bool PADR = CS_ROW_PAD && !ILV && (B == 1 || LD % 32 == 0) && Q % 32 == 0;
  if constexpr (ILV) {
    const unsigned base = j * B + b;
#pragma unroll
    for (int r = 0; r < 8; ++r) v[r] = buf[lp(base + r * Q * B)];
  } else if constexpr (PADR) {
    const unsigned base = b * prc(LD) + lpr(j);
#pragma unroll
    for (int r = 0; r < 8; ++r) v[r] = buf[base + prc(r * Q)];
  } else {
#pragma unroll
    for (int r = 0; r < 8; ++r) v[r] = buf[lds_addr<ILV, B, LD>(b, j + r * Q)];
  }
  // twiddles W_L^{r j}: W^j and W^{4j} from the table, the rest by products
  float2 w[8];
  w[1] = tw[j];
  w[2] = cmul(w[1], w[1]);
  w[3] = cmul(w[2], w[1]);
  w[4] = tw[4 * j];
  w[5] = cmul(w[4], w[1]);
  w[6] = cmul(w[4], w[2]);
  w[7] = cmul(w[4], w[3]);
#pragma unroll
  for (int r = 1; r < 8; ++r) v[r] = INV ? cmulc(v[r], w[r]) : cmul(v[r], w[r]);
  dft8<INV>(v);
}

#ifndef CS_MID_RADIX16
#define CS_MID_RADIX16 1
#endif
template <int L, int B, int T, bool INV, bool ILV, int LD, int NS = 8>
__device__ __forceinline__ void lds_fft_mid(float2* __restrict__ buf, const float2* __restrict__ tw,
                                            unsigned tid) {
  if constexpr (NS < L / 8) {
    // radix 8 (radix 16 when exactly 16 remains: one LDS round trip instead
    // of two), with one radix-4 or radix-2 stage for the remaining factor
    constexpr int p = ilog2c(L / (8 * NS));
    constexpr int R = (p == 4 && CS_MID_RADIX16) ? 16 : (p % 3 == 0) ? 8 : ((p % 3 == 2) ? 4 : (p == 1 ? 2 : 4));
    stockham_stage<L, B, T, INV, ILV, LD, NS, R>(buf, tw, tid);
    lds_fft_mid<L, B, T, INV, ILV, LD, NS * R>(buf, tw, tid);
  }
}

}  // namespace cs
