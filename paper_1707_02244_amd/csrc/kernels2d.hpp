// 2-D path: an R x C real image (row-major), sensing A = P G with G the
// periodic 2-D convolution by g = s * h (sensing kernel s, blur h; the blur
// as a circulant is the device of Section 7) and P keeping pixels (2i, 2j).
// The 2-D DFT diagonalises G with eigenvalues g_hat = DFT2(s) DFT2(h).
//
// Packing: z[r][j] = x[r][2j] + i x[r][2j+1], j < H = C/2.  With
// Z = DFT2(z) (R x H) and w = W_C^{k2}:
//   E = (Z[k1][k2] + conj Z[-k1][-k2]) / 2,  O = -i (Z[k1][k2] - conj Z[-k1][-k2]) / 2,
//   X[k1][k2] = E + w O,   X[k1][k2 + H] = E - w O.
//
// Row pass ("time side"): a workgroup owns kRows2 = 8 image rows and runs
// H-point FFTs along them.  The row-transformed image is stored transposed
// with each mirror column pair interleaved: T[w][r][s] holds column k2 = w
// (s = 0) and its mirror H - w (s = 1; pair 0 holds columns 0 and H/2).  The
// column pass then reads one contiguous block per workgroup and the row pass
// 128-byte runs (8 rows x the two columns of a pair).  The time-domain steps (soft threshold, Eq. 4;
// ADMM's z and u updates, Alg. 2) run between the inverse and the forward
// row transforms.
//
// Column pass ("frequency side"): workgroup w owns packed columns p = w and
// H - w (workgroup 0: columns 0 and H/2, each its own mirror).  R-point FFTs
// along both give Z; each decimation class of the m1 x m2 = R/2 x H grid,
//   {(k1' + l1 R/2, p + l2 H) : l1, l2 in {0, 1}},
// takes its four bins from rows k1', k1' + R/2 of column p and rows -k1',
// R/2 - k1' of column H - p, and the same four values also carry the mirror
// class (-k1', -p), so every update is local to the workgroup.
//
// Per class, with S = (1/4) sum_l g_l X_l the m-point DFT of A x (P folds
// the four bins) and Lam = (1/4) sum_l |g_l|^2 the eigenvalue of A A^T:
//   ISTA (Alg. 1):  step_l = conj(g_l) tau (Y_hat - S)       (DFT of tau A^T r)
//   ADMM (Alg. 2), x-update from W = DFT(z - u):
//       X'_l = W_l + conj(g_l) (Y_hat - S_W) / (rho + Lam),
//   which equals the Woodbury form (Q - conj(g) T)/rho with
//   Q = conj(g) Y_hat + rho W and T = sum g Q / (4 rho + sum |g|^2), without
//   its cancellation: with an unscaled +-1 sensing kernel Lam reaches ~1e7
//   rho, and forming Q and subtracting conj(g) T would leave no correct FP32
//   digit in the data-fit component.
#pragma once
#include "kernels.hpp"

namespace cs {

#ifndef CS_ROWS2
#define CS_ROWS2 8
#endif
#ifndef CS_COL2_MINW
#define CS_COL2_MINW 1   // column pass: minimum waves per SIMD the compiler must allow
#endif
#ifndef CS_COL2_MINW_LARGE
// column pass with 512 threads (R >= 2048): 4 waves per SIMD (at most 128
// VGPRs) lets two workgroups share a CU, so one workgroup's loads and stores
// overlap the other's FFT stages (4096 x 4096 ADMM column pass 76.5 -> 63.4
// us, with 16 VGPRs spilled)
#define CS_COL2_MINW_LARGE 4
#endif
#ifndef CS_C2_LATE_G
#define CS_C2_LATE_G 1   // column pass: class operands loaded after the forward transform
#endif
#ifndef CS_ROW2_MINW
#define CS_ROW2_MINW 1   // row pass: same
#endif
#ifndef CS_ROW2_TWLDS
#define CS_ROW2_TWLDS 1  // row pass: FFT twiddles staged in LDS (else read from the global table)
#endif
constexpr int kRows2 = CS_ROWS2;   // image rows per row-pass workgroup (8: 64-byte runs of T)
constexpr int kPad2 = CS_ROW_PAD ? 0 : 4;   // float2 padding between LDS rows / columns

enum OpC2 : int {
  C2_ISTA = 0,     // ISTA class update (step spectrum)
  C2_ADMM = 1,     // ADMM x-update from DFT(z - u)
  C2_RES = 2,      // objective trace only: sum |Y_hat - S|^2 of the input
  C2_MUL = 3,      // X -> g_hat X            (G x)
  C2_MULC = 4,     // X -> conj(g_hat) X      (G^T x)
  C2_SPEC = 5,     // write X to the g-table layout
  C2_SPECMUL = 6,  // multiply the g-table by X
  C2_YHAT = 7,     // write X(k1, p), k1 < R/2, to the y-table layout
};

enum ModeR2 : int {
  R2_FWD_REAL = 0,  // image -> forward -> T
  R2_FWD_UP = 1,    // P^T y (y: R/2 x H) -> forward -> T
  R2_FWD_ZMU = 2,   // z - u -> forward -> T
  R2_ISTA = 3,      // T (step) -> inverse -> x += step, threshold -> forward -> T
  R2_ADMM = 4,      // T -> inverse (x) -> z, u update -> forward(z - u) -> T
  R2_OUT_ALL = 5,   // T -> inverse -> image
  R2_OUT_DEC = 6,   // T -> inverse -> pixels (2i, 2j)
};

struct Col2Args {
  float2* T;               // [H/2][R][2]: column pairs {w, H - w} ({0, H/2} for w = 0)
  const float2* G;         // g_hat: [H/2 + 1][2][R], G[p][l2][k1] = g_hat(k1, p + l2 H)
  const float2* Yt;        // Y_hat: [H/2 + 1][R/2], Yt[p][k1'] = Y_hat(k1', p)
  float2* table;           // C2_SPEC / C2_SPECMUL (G layout), C2_YHAT (Yt layout)
  const float2* twR;       // W_R^e, e < R
  const float2* twc;       // W_C^p, p <= H/2
  int H;
  float inv_n;             // 1 / (R C): the split's 1/2 times the inverse's 1/(R H)
  float tau;               // ISTA step
  float rho;               // ADMM penalty
  double* res;             // objective trace: per-workgroup sum of weight * |Y_hat - S|^2
};

struct Row2Args {
  float2* T;               // [H/2][R][2], as in Col2Args
  const float2* twH;       // W_H^e, e < H
  int R;
  int H;
  const float* in0;        // R2_FWD_REAL: image; R2_FWD_UP: y; R2_FWD_ZMU: z
  const float* in1;        // R2_FWD_ZMU: u
  float* out0;             // R2_ADMM last: x; R2_OUT_*: output
  float* out1;             // R2_ADMM last: z
  float* u;                // state: ISTA x, ADMM u
  float thr;               // ISTA tau * lambda, ADMM lambda / rho
  int last;                // final iteration: no forward transform
  double* l1;              // objective trace: per-workgroup sum |x|
};

#ifndef CS_COL2_T
#define CS_COL2_T 512    // column-pass threads for R >= 2048
#endif
#ifndef CS_ROW2_T
#define CS_ROW2_T 512    // row-pass threads for 8 H >= 8192
#endif
template <int R>
constexpr int col2_threads() { return R >= 2048 ? CS_COL2_T : 256; }
template <int R>
constexpr int col2_minw() { return R >= 2048 ? CS_COL2_MINW_LARGE : CS_COL2_MINW; }
template <int H>
constexpr int row2_threads() { return kRows2 * H >= 8192 ? CS_ROW2_T : 256; }

// ---------------------------------------------------------------------------
// Column pass (frequency side).
template <int R, int OP>
__global__ __launch_bounds__(col2_threads<R>(), col2_minw<R>()) void k2_col(Col2Args a) {
  constexpr int T = col2_threads<R>();
  constexpr int LD = R + kPad2;
  constexpr int NE = 2 * R;
  constexpr int EPT = (NE + T - 1) / T;
  constexpr bool TW_LDS = (lds_rows(2 * LD) + R) * 8 <= 64 * 1024;
  constexpr bool GROUP = (OP == C2_ISTA || OP == C2_ADMM || OP == C2_RES);
  constexpr bool TABLE = (OP == C2_SPEC || OP == C2_SPECMUL || OP == C2_YHAT);
  constexpr bool WRITE_BACK = (OP == C2_ISTA || OP == C2_ADMM || OP == C2_MUL || OP == C2_MULC);
  constexpr int HR = R / 2;
  __shared__ float2 lds[lds_rows(2 * LD)];
  __shared__ float2 tws_l[TW_LDS ? R : 1];
  const unsigned tid = threadIdx.x;
  const int w = blockIdx.x;
  const int H = a.H;
  const int col0 = w, col1 = w ? (H - w) : (H >> 1);
  const float2* tws = TW_LDS ? tws_l : a.twR;

  float2 v[EPT];
#pragma unroll
  for (int k = 0; k < EPT; ++k) {
    const unsigned i = tid + k * T;
    if (NE % T == 0 || i < NE) v[k] = a.T[(size_t)w * NE + i];   // element (r = i/2, slot i%2)
  }
  // group operands: g_hat at the class's four bins, Y_hat of the class.
  // Loaded with the column (early) or after the forward transform (late:
  // they are then not live across it, which keeps the R = 4096 pass within
  // 128 VGPRs without spills)
  constexpr int NGMAX = HR;   // groups per workgroup (w > 0); workgroup 0 has R/2 + 2
  constexpr int GPT = GROUP ? (NGMAX + 2 + T - 1) / T : 1;
  constexpr bool LATE_G = CS_C2_LATE_G && GPT > 2;
  const int ng = w ? HR : 2 * (R / 4 + 1);
  float2 gg[GPT][4], gy[GPT];
  auto load_groups = [&]() __attribute__((always_inline)) {
#pragma unroll
    for (int k = 0; k < GPT; ++k) {
      const int g = tid + k * T;
      if (g < ng) {
        const int slot = w ? 0 : g / (R / 4 + 1);
        const int k1 = w ? g : g % (R / 4 + 1);
        const int p = slot ? col1 : col0;
        const float2* gp = a.G + (size_t)p * 2 * R;
        gg[k][0] = gp[k1];
        gg[k][1] = gp[k1 + HR];
        gg[k][2] = gp[R + k1];
        gg[k][3] = gp[R + k1 + HR];
        gy[k] = a.Yt[(size_t)p * HR + k1];
      }
    }
  };
  if constexpr (GROUP && !LATE_G) load_groups();
  if constexpr (TW_LDS) {
    for (unsigned i = tid; i < R; i += T) tws_l[i] = a.twR[i];
  }
#pragma unroll
  for (int k = 0; k < EPT; ++k) {
    const unsigned i = tid + k * T;
    if (NE % T == 0 || i < NE) lds[lpr((i & 1) * LD + (i >> 1))] = v[k];
  }
  __syncthreads();
  lds_fft<R, 2, T, false, false, LD>(lds, tws, tid);

  float res_acc = 0.0f;
  if constexpr (GROUP) {
    if constexpr (LATE_G) load_groups();
#pragma unroll
    for (int k = 0; k < GPT; ++k) {
      const int g = tid + k * T;
      if (g >= ng) continue;
      const int slot = w ? 0 : g / (R / 4 + 1);
      const int k1 = w ? g : g % (R / 4 + 1);
      const int sa = slot, sb = w ? 1 : slot;
      const bool self = (w == 0) && (k1 == 0 || k1 == R / 4);
      const float2 wp = a.twc[slot ? (H >> 1) : w];
      const int a0 = k1, a1 = k1 + HR, b0 = (R - k1) & (R - 1), b1 = HR - k1;
      const float2 za0 = lds[lpr(sa * LD + a0)], za1 = lds[lpr(sa * LD + a1)];
      const float2 zb0 = cconj(lds[lpr(sb * LD + b0)]), zb1 = cconj(lds[lpr(sb * LD + b1)]);
      const float2 E0 = cscale(cadd(za0, zb0), 0.5f), O0 = cscale(cmulmi(csub(za0, zb0)), 0.5f);
      const float2 E1 = cscale(cadd(za1, zb1), 0.5f), O1 = cscale(cmulmi(csub(za1, zb1)), 0.5f);
      const float2 wO0 = cmul(wp, O0), wO1 = cmul(wp, O1);
      // bins (k1, p), (k1 + R/2, p), (k1, p + H), (k1 + R/2, p + H)
      float2 X[4] = {cadd(E0, wO0), cadd(E1, wO1), csub(E0, wO0), csub(E1, wO1)};
      float2 S = c2(0.f, 0.f);
#pragma unroll
      for (int l = 0; l < 4; ++l) S = cadd(S, cmul(gg[k][l], X[l]));
      S = cscale(S, 0.25f);
      const float2 r = csub(gy[k], S);
      const float wt = self ? 1.0f : 2.0f;
      if constexpr (OP == C2_RES) {
        res_acc += wt * cabs2(r);
        continue;
      } else if constexpr (OP == C2_ISTA) {
        res_acc += wt * cabs2(r);
        const float2 E = cscale(r, a.tau);
#pragma unroll
        for (int l = 0; l < 4; ++l) X[l] = cconjmul(gg[k][l], E);
      } else {
        float lam = 0.0f;
#pragma unroll
        for (int l = 0; l < 4; ++l) lam += cabs2(gg[k][l]);
        const float2 E = cscale(r, 1.0f / (a.rho + 0.25f * lam));
#pragma unroll
        for (int l = 0; l < 4; ++l) X[l] = cadd(X[l], cconjmul(gg[k][l], E));
        if (a.res) {
          float2 S1 = c2(0.f, 0.f);
#pragma unroll
          for (int l = 0; l < 4; ++l) S1 = cadd(S1, cmul(gg[k][l], X[l]));
          res_acc += wt * cabs2(csub(gy[k], cscale(S1, 0.25f)));
        }
      }
      // inverse split, scaled by 1/(R C)
      const float2 Ea = cscale(cadd(X[0], X[2]), a.inv_n), Oa = cscale(cmulc(csub(X[0], X[2]), wp), a.inv_n);
      const float2 Eb = cscale(cadd(X[1], X[3]), a.inv_n), Ob = cscale(cmulc(csub(X[1], X[3]), wp), a.inv_n);
      lds[lpr(sa * LD + a0)] = cadd(Ea, cmuli(Oa));
      lds[lpr(sa * LD + a1)] = cadd(Eb, cmuli(Ob));
      if (!self) {
        lds[lpr(sb * LD + b0)] = cconj(csub(Ea, cmuli(Oa)));
        lds[lpr(sb * LD + b1)] = cconj(csub(Eb, cmuli(Ob)));
      }
    }
    if (a.res) {
      const double s = block_sum<T>(double(res_acc), tid);
      if (tid == 0) a.res[w] = s;
    }
  } else {
    // pointwise modes, by split pairs (k1, p) / (-k1, -p).  Table modes only
    // read LDS and visit every k1 of both columns of workgroup 0; in-place
    // modes visit k1 <= R/2 there (k1 = 0 and R/2 pair with themselves).
    const int ni = w ? R : (TABLE ? 2 * R : 2 * (HR + 1));
    const int per = TABLE ? R : (HR + 1);
    for (int q = tid; q < ni; q += T) {
      const int slot = w ? 0 : q / per;
      const int k1 = w ? q : q % per;
      const int sa = slot, sb = w ? 1 : slot;
      const int p = slot ? (H >> 1) : w;
      const int b = (R - k1) & (R - 1);
      const bool self = (w == 0) && (k1 == 0 || k1 == HR);
      const float2 wp = a.twc[p];
      const float2 za = lds[lpr(sa * LD + k1)], zbc = cconj(lds[lpr(sb * LD + b)]);
      const float2 E = cscale(cadd(za, zbc), 0.5f), O = cscale(cmulmi(csub(za, zbc)), 0.5f);
      const float2 wO = cmul(wp, O);
      const float2 Xlo = cadd(E, wO), Xhi = csub(E, wO);
      float2* tp = a.table + (size_t)p * 2 * R;
      if constexpr (OP == C2_SPEC) {
        tp[k1] = Xlo;
        tp[R + k1] = Xhi;
      } else if constexpr (OP == C2_SPECMUL) {
        tp[k1] = cmul(tp[k1], Xlo);
        tp[R + k1] = cmul(tp[R + k1], Xhi);
      } else if constexpr (OP == C2_YHAT) {
        if (k1 < HR) a.table[(size_t)p * HR + k1] = Xlo;
      } else {
        const float2* gp = a.G + (size_t)p * 2 * R;
        const float2 glo = gp[k1], ghi = gp[R + k1];
        const float2 Vlo = OP == C2_MUL ? cmul(glo, Xlo) : cconjmul(glo, Xlo);
        const float2 Vhi = OP == C2_MUL ? cmul(ghi, Xhi) : cconjmul(ghi, Xhi);
        const float2 E_ = cscale(cadd(Vlo, Vhi), a.inv_n);
        const float2 O_ = cscale(cmulc(csub(Vlo, Vhi), wp), a.inv_n);
        lds[lpr(sa * LD + k1)] = cadd(E_, cmuli(O_));
        if (!self) lds[lpr(sb * LD + b)] = cconj(csub(E_, cmuli(O_)));
      }
    }
  }
  if constexpr (WRITE_BACK) {
    __syncthreads();
    lds_fft<R, 2, T, true, false, LD>(lds, tws, tid);
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
      const unsigned i = tid + k * T;
      if (NE % T == 0 || i < NE) a.T[(size_t)w * NE + i] = lds[lpr((i & 1) * LD + (i >> 1))];
    }
  }
}

// ---------------------------------------------------------------------------
// Row pass (time side): workgroup b owns image rows [8b, 8b + 8).
template <int H, int MODE>
__global__ __launch_bounds__(row2_threads<H>(), CS_ROW2_MINW) void k2_row(Row2Args a) {
  constexpr int T = row2_threads<H>();
  constexpr int RW = kRows2;
  constexpr int LD = H + kPad2;
  constexpr int NE = RW * H;
  constexpr int EPT = (NE + T - 1) / T;
  constexpr int CH = EPT < 8 ? EPT : 8;
  constexpr bool FULL = (NE % T) == 0;
  constexpr bool HAS_INV = (MODE == R2_ISTA || MODE == R2_ADMM || MODE == R2_OUT_ALL || MODE == R2_OUT_DEC);
  __shared__ float2 lds[lds_rows(RW * LD)];
  __shared__ float2 tws_l[CS_ROW2_TWLDS ? H : 1];
  const float2* tws = CS_ROW2_TWLDS ? tws_l : a.twH;
  const unsigned tid = threadIdx.x;
  const int r0 = blockIdx.x * RW;
  const int R = a.R;
  const size_t tbase = (size_t)r0 * H;   // first packed element of the rows (time side)
  // spectral side, element i of the block in T order: pair w = i / (2 RW),
  // row c = (i / 2) % RW, side s = i % 2 (column w, or its mirror)
  auto t_off = [&](unsigned i) -> size_t {
    return ((size_t)(i / (2 * RW)) * R + r0 + (i / 2) % RW) * 2 + (i & 1);
  };
  auto t_lds = [&](unsigned i) -> unsigned {
    const unsigned w = i / (2 * RW), c = (i / 2) % RW;
    const unsigned k2 = (i & 1) ? (w ? H - w : (H >> 1)) : w;
    return c * LD + k2;
  };
  if (CS_ROW2_TWLDS)
    for (unsigned i = tid; i < H; i += T) tws_l[i] = a.twH[i];

  if constexpr (HAS_INV) {
    // T[w][r0 + c][s] -> lds[c][k2]: 128-byte runs (8 rows x 2 columns)
#pragma unroll
    for (int k0 = 0; k0 < EPT; k0 += CH) {
      float2 v[CH];
#pragma unroll
      for (int k = 0; k < CH; ++k) {
        const unsigned i = tid + (k0 + k) * T;
        if (FULL || i < NE) v[k] = a.T[t_off(i)];
      }
#pragma unroll
      for (int k = 0; k < CH; ++k) {
        const unsigned i = tid + (k0 + k) * T;
        if (FULL || i < NE) lds[lpr(t_lds(i))] = v[k];
      }
    }
    __syncthreads();
    lds_fft<H, RW, T, true, false, LD>(lds, tws, tid);
    bool fwd = true;
    if constexpr (MODE == R2_ISTA || MODE == R2_ADMM) {
      float2* st = reinterpret_cast<float2*>(a.u) + tbase;
      float l1_acc = 0.0f;
#pragma unroll
      for (int k0 = 0; k0 < EPT; k0 += CH) {
        float2 sv[CH];
#pragma unroll
        for (int k = 0; k < CH; ++k) {
          const unsigned i = tid + (k0 + k) * T;
          if (FULL || i < NE) sv[k] = st[i];
        }
#pragma unroll
        for (int k = 0; k < CH; ++k) {
          const unsigned i = tid + (k0 + k) * T;
          if (FULL || i < NE) {
            const unsigned li = (i / H) * LD + (i % H);
            if constexpr (MODE == R2_ISTA) {
              const float2 vv = cadd(sv[k], lds[lpr(li)]);
              const float2 x = c2(soft(vv.x, a.thr), soft(vv.y, a.thr));
              l1_acc += fabsf(x.x) + fabsf(x.y);
              st[i] = x;
              lds[lpr(li)] = x;
            } else {
              const float2 x = lds[lpr(li)];
              l1_acc += fabsf(x.x) + fabsf(x.y);
              const float2 xu = cadd(x, sv[k]);
              const float2 z = c2(soft(xu.x, a.thr), soft(xu.y, a.thr));
              const float2 u1 = csub(xu, z);
              st[i] = u1;
              if (a.last) {
                reinterpret_cast<float2*>(a.out0)[tbase + i] = x;
                reinterpret_cast<float2*>(a.out1)[tbase + i] = z;
              } else {
                lds[lpr(li)] = csub(z, u1);
              }
            }
          }
        }
      }
      if (a.l1) {
        const double s = block_sum<T>(double(l1_acc), tid);
        if (tid == 0) a.l1[blockIdx.x] = s;
      }
      fwd = !a.last;
    } else if constexpr (MODE == R2_OUT_ALL) {
      for (unsigned i = tid; i < NE; i += T)
        reinterpret_cast<float2*>(a.out0)[tbase + i] = lds[lpr((i / H) * LD + (i % H))];
      fwd = false;
    } else {  // R2_OUT_DEC: even rows, even columns (the real parts)
      for (unsigned i = tid; i < NE; i += T) {
        const unsigned c = i / H, j = i % H;
        const int r = r0 + int(c);
        if ((r & 1) == 0) a.out0[(size_t)(r >> 1) * H + j] = lds[lpr(c * LD + j)].x;
      }
      fwd = false;
    }
    if (!fwd) return;
    __syncthreads();
  } else {
#pragma unroll
    for (int k0 = 0; k0 < EPT; k0 += CH) {
      float2 v[CH];
#pragma unroll
      for (int k = 0; k < CH; ++k) {
        const unsigned i = tid + (k0 + k) * T;
        if (FULL || i < NE) {
          if constexpr (MODE == R2_FWD_REAL) {
            v[k] = reinterpret_cast<const float2*>(a.in0)[tbase + i];
          } else if constexpr (MODE == R2_FWD_UP) {
            const int r = r0 + int(i / H);
            v[k] = c2((r & 1) == 0 ? a.in0[(size_t)(r >> 1) * H + (i % H)] : 0.0f, 0.0f);
          } else {
            v[k] = csub(reinterpret_cast<const float2*>(a.in0)[tbase + i],
                        reinterpret_cast<const float2*>(a.in1)[tbase + i]);
          }
        }
      }
#pragma unroll
      for (int k = 0; k < CH; ++k) {
        const unsigned i = tid + (k0 + k) * T;
        if (FULL || i < NE) lds[lpr((i / H) * LD + (i % H))] = v[k];
      }
    }
    __syncthreads();
  }
  lds_fft<H, RW, T, false, false, LD>(lds, tws, tid);
#pragma unroll
  for (int k = 0; k < EPT; ++k) {
    const unsigned i = tid + k * T;
    if (FULL || i < NE) a.T[t_off(i)] = lds[lpr(t_lds(i))];
  }
}

}  // namespace cs
