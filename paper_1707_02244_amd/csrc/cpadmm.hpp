// Circulant ADMM with an arbitrary row set (Section 4.3, Alg. 3).
//
// A = P C with C circulant (first column c) and P keeping the rows in an
// arbitrary set Omega of m indices.  The LASSO is split as
//     min 1/2 ||y - P v||^2 + alpha ||z||_1   s.t.  v = C x,  z = x,
// and each iteration of the augmented-Lagrangian method (scaled multipliers
// mu for v = C x, nu for z = x) is
//     x  = B (rho C^T (v + mu) + sigma (z - nu)),   B = (rho C^T C + sigma I)^-1
//     v  = D (rho C x - rho mu + P^T y),             D = (P^T P + rho I)^-1
//     z  = eta_{alpha/sigma}(x + nu)
//     mu = mu + tau (v - C x),   nu = nu + tau (x - z).
// B and C^T C are circulant, so the x-update and C x are one pointwise step
// in the Fourier domain:  X = (rho conj(c_hat) A + sigma B_) / (rho |c_hat|^2 +
// sigma) with A, B_ the spectra of a = v + mu and b = z - nu, and C x has the
// spectrum c_hat X.  D is diagonal (1/(1 + rho) on Omega, 1/rho elsewhere):
// the v-update is pointwise in the time domain.
//
// Two real signals travel through the four-step transform together (the
// packed real layout of kernels.hpp, N = n/2 complex points, N = N1 * N2):
//   column pass (time side): inverse column FFTs of the spectra of x and C x,
//     the v, z, mu, nu updates, forward column FFTs of a and b;
//   row pass (frequency side): forward row FFTs of a and b, the real split,
//     the per-bin update above for bins k and N - k, the inverse split of X
//     and c_hat X, inverse row FFTs.
// Layouts, chosen so that both passes move whole 128-byte runs:
//   - one spectrum buffer Yab for both signals (a in / x out, b in / C x
//     out), interleaving each mirror row pair and the two signals:
//     element (signal g, row k1, column j2) at Yab[((w N2 + j2) 2 + g) 2 + s]
//     with pair w = min(k1, N1 - k1) and side s = (k1 != w) (pair 0 holds
//     rows 0 and N1/2).  A row-pass workgroup reads one contiguous block;
//     a column-pass workgroup of CB columns reads 4 CB contiguous values per
//     pair.
//   - the time-domain state of a solve (mu, nu, P^T y and the indicator of
//     Omega) in column blocks: sample pair i N2 + j2 at [(b N1 + i) CB + c],
//     b = j2 / CB, c = j2 mod CB, so each column-pass workgroup owns one
//     contiguous range.  The last column pass writes x, v, z, mu and nu in
//     natural order into the caller's arrays.
#pragma once
#include "kernels.hpp"

namespace cs {

struct CpArgs {
  float2* Yab;             // [N1/2][N2][2][2] four-step buffer of a / x and b / C x
  const float2* chat;      // c_hat table ([k1*N2 + k2], Nyquist at [N])
  const float2* twk1;      // W_n^{k1}
  const float2* twp;       // W_{2 N2}^p
  const float2* twlo;      // W_N^e, e < 2^lo_bits
  const float2* twhi;      // W_N^{e * 2^lo_bits}
  const float2* tw1;       // W_{N1}^e
  const float2* tw2;       // W_{N2}^e
  int lo_bits;
  int N1, N2, N;
  float inv_n;
  float rho, sigma, tau, thr;   // thr = alpha / sigma
  float d_in, d_out;            // D on Omega (1 / (1 + rho)) and elsewhere (1 / rho)
  float2* mu_b;            // mu, column-blocked (n/2 pairs)
  float2* nu_b;            // nu, column-blocked
  const float2* py_b;      // P^T y, column-blocked
  const float2* om_b;      // indicator of Omega, column-blocked
  float* mu;               // outputs in natural order, written by the last
  float* nu;               //   column pass
  float* v;
  float* z;
  float* x;
};

__device__ __forceinline__ float2 cp_twN(const CpArgs& a, int e) {
  e &= (a.N - 1);
  return cmul(a.twlo[e & ((1 << a.lo_bits) - 1)], a.twhi[e >> a.lo_bits]);
}

// Row-pass threads: 512 for rows of 1024 points and more (16 values per
// thread), else 256.
constexpr int cp_row_threads(int N2) { return N2 >= 1024 ? 512 : 256; }

// Row pass of row pair w: LDS slots 0, 1 = rows {w, N1 - w} of a, slots 2, 3
// = the same rows of b ({0, N1/2} for w = 0); slot g 2 + s is element
// (j2, g, s) of the pair's contiguous block of Yab.  The FFT twiddles are
// staged in LDS only where two workgroups still fit on a CU with them
// (N2 <= 1024); longer rows read them from the global table.
template <int N2, int T>
__global__ __launch_bounds__(T, 2) void k_cp_row(CpArgs a) {
  constexpr int LD = N2 + kPadA;
  constexpr int NR = 4 * N2;
  constexpr int EPT = (NR + T - 1) / T;
  constexpr bool TWL = (lds_rows(4 * LD) + N2) * 8 <= 80 * 1024;
  static_assert(lds_rows(4 * LD) * 8 <= 80 * 1024, "row pass exceeds its LDS budget");
  __shared__ float2 lds[lds_rows(4 * LD)];
  __shared__ float2 tws_l[TWL ? N2 : 1];
  const float2* tws = TWL ? tws_l : a.tw2;
  const unsigned tid = threadIdx.x;
  const int w = blockIdx.x;
  const int N1 = a.N1;
  float2* blk = a.Yab + (size_t)w * (4 * N2);
  if constexpr (TWL)
    for (int i = tid; i < N2; i += T) tws_l[i] = a.tw2[i];
  float2 rv[EPT];
#pragma unroll
  for (int k = 0; k < EPT; ++k) {
    const int i = tid + k * T;
    if (NR % T == 0 || i < NR) rv[k] = blk[i];
  }
#pragma unroll
  for (int k = 0; k < EPT; ++k) {
    const int i = tid + k * T;
    if (NR % T == 0 || i < NR) lds[lpr((i & 3) * LD + (i >> 2))] = rv[k];
  }
  __syncthreads();
  lds_fft<N2, 4, T, false, false, LD>(lds, tws, tid);

  // split pairs (k, N - k): w > 0: slot 0 position p with slot 1 position
  // N2-1-p; w = 0: row 0 positions p in [0, N2/2] with (N2 - p) mod N2, row
  // N1/2 positions p < N2/2 with N2-1-p
  const int np = w ? N2 : (N2 + 1);
  for (int g = tid; g < np; g += T) {
    int sa, sb, rowa, p, mode;
    if (w) { sa = 0; sb = 1; rowa = w; p = g; mode = 0; }
    else if (g <= (N2 >> 1)) { sa = 0; sb = 0; rowa = 0; p = g; mode = 1; }
    else { sa = 1; sb = 1; rowa = N1 >> 1; p = g - (N2 >> 1) - 1; mode = 2; }
    const int rowb = (mode == 0) ? (N1 - w) : rowa;
    const int q = (mode == 1) ? ((N2 - p) & (N2 - 1)) : (N2 - 1 - p);
    const bool write_b = !(mode == 1 && (p == 0 || p == (N2 >> 1)));
    const float2 wt = cmul(a.twk1[rowa], a.twp[p]);
    // real-signal bins k (index a) and N - k (index b) of the packed signal
    // in slots (s0 + sa, s0 + sb)
    auto split = [&](int s0, float2& Xk, float2& Xnk) {
      const float2 za = lds[lpr((s0 + sa) * LD + p)];
      const float2 zbc = cconj(lds[lpr((s0 + sb) * LD + q)]);
      const float2 P = cscale(cadd(za, zbc), 0.5f);
      const float2 Q = cscale(cmulmi(csub(za, zbc)), 0.5f);
      const float2 wq = cmul(wt, Q);
      Xk = cadd(P, wq);
      Xnk = cconj(csub(P, wq));
    };
    // inverse split of bins (k, N - k) into the packed slots, with 1/n
    auto unsplit = [&](int s0, float2 Va, float2 Vb) {
      const float2 vbc = cconj(Vb);
      const float2 E_ = cscale(cadd(Va, vbc), a.inv_n);
      const float2 O_ = cscale(cmulc(csub(Va, vbc), wt), a.inv_n);
      lds[lpr((s0 + sa) * LD + p)] = cadd(E_, cmuli(O_));
      if (write_b) lds[lpr((s0 + sb) * LD + q)] = cconj(csub(E_, cmuli(O_)));
    };
    float2 Ak, Ank, Bk, Bnk;
    split(0, Ak, Ank);
    split(2, Bk, Bnk);
    const float2 ck = a.chat[(size_t)rowa * N2 + p];
    const float2 cnk = (mode == 1 && p == 0) ? a.chat[a.N] : a.chat[(size_t)rowb * N2 + q];
    // X = (rho conj(c) A + sigma B) / (rho |c|^2 + sigma)
    const float2 Xk = cscale(cadd(cscale(cconjmul(ck, Ak), a.rho), cscale(Bk, a.sigma)),
                             1.0f / fmaf(a.rho, cabs2(ck), a.sigma));
    const float2 Xnk = cscale(cadd(cscale(cconjmul(cnk, Ank), a.rho), cscale(Bnk, a.sigma)),
                              1.0f / fmaf(a.rho, cabs2(cnk), a.sigma));
    unsplit(0, Xk, Xnk);
    unsplit(2, cmul(ck, Xk), cmul(cnk, Xnk));
  }
  __syncthreads();
  lds_fft<N2, 4, T, true, false, LD>(lds, tws, tid);
#pragma unroll
  for (int k = 0; k < EPT; ++k) {
    const int i = tid + k * T;
    if (NR % T == 0 || i < NR) blk[i] = lds[lpr((i & 3) * LD + (i >> 2))];
  }
}

// Column pass on CB adjacent columns [CB b, CB b + CB): LDS holds the columns
// of x (sequences 0 .. CB-1) and of C x (CB .. 2CB-1) interleaved, element
// (sequence s, index i) at [i * 2CB + s].  The workgroup's part of Yab is
// 4 CB contiguous values per row pair: value r of pair w is column
// j2 = CB b + r / 4 of signal (r / 2) mod 2, row w (r even) or its mirror.
// LAST: write x, v, z, mu, nu in natural order and skip the forward
// transforms.
template <int N1, int CB, int T, bool LAST>
__global__ __launch_bounds__(T, 2) void k_cp_col(CpArgs a) {
  constexpr int S = 2 * CB;
  constexpr int NE = N1 * S;
  constexpr int EPT = (NE + T - 1) / T;
  constexpr bool FULL = NE % T == 0;
  __shared__ float2 lds[lds_padded(NE)];
  __shared__ float2 tws[N1];
  const unsigned tid = threadIdx.x;
  const int j2_0 = blockIdx.x * CB;
  const int N2 = a.N2;
  for (int i = tid; i < N1; i += T) tws[i] = a.tw1[i];
  // element e of the workgroup's part of Yab: its global offset, its LDS
  // slot and its four-step twiddle exponent j2 * k1
  auto gaddr = [&](int e, size_t& gofs, int& li, int& ex) {
    const int w = e / (4 * CB), r = e % (4 * CB);
    const int c = r >> 2, g = (r >> 1) & 1;
    const int k1 = (r & 1) ? (w ? N1 - w : (N1 >> 1)) : w;
    gofs = ((size_t)w * N2 + j2_0) * 4 + r;
    li = k1 * S + g * CB + c;
    ex = (j2_0 + c) * k1;
  };
  // loads in chunks of CH per thread (all of a chunk in flight at once)
  constexpr int CH = EPT < 8 ? EPT : 8;
#pragma unroll 1
  for (int k0 = 0; k0 < EPT; k0 += CH) {
    float2 v[CH], t[CH];
    int l[CH];
#pragma unroll
    for (int k = 0; k < CH; ++k) {
      const int e = tid + (k0 + k) * T;
      if (FULL || e < NE) {
        size_t go;
        int ex;
        gaddr(e, go, l[k], ex);
        v[k] = a.Yab[go];
        t[k] = cp_twN(a, ex);
      }
    }
#pragma unroll
    for (int k = 0; k < CH; ++k) {
      const int e = tid + (k0 + k) * T;
      if (FULL || e < NE) lds[lp(l[k])] = cmulc(v[k], t[k]);
    }
  }
  __syncthreads();
  lds_fft<N1, S, T, true, true, N1>(lds, tws, tid);
  // time domain: x at [i*S + c], C x at [i*S + CB + c]; sample pair
  // i*N2 + j2_0 + c, blocked state index blockIdx.x * N1 * CB + q
  const size_t qb0 = (size_t)blockIdx.x * N1 * CB;
#pragma unroll 2
  for (int q = tid; q < N1 * CB; q += T) {
    const int i = q / CB, c = q % CB;
    const float2 x = lds[lp(i * S + c)];
    const float2 cx = lds[lp(i * S + CB + c)];
    const size_t qb = qb0 + q;
    const float2 m0 = a.mu_b[qb], n0 = a.nu_b[qb], py = a.py_b[qb], om = a.om_b[qb];
    auto upd = [&](float xe, float cxe, float me, float ne, float pye, float ome, float& ve, float& ze, float& me1,
                   float& ne1) {
      const float dd = ome != 0.0f ? a.d_in : a.d_out;
      ve = dd * (a.rho * cxe - a.rho * me + pye);
      ze = soft(xe + ne, a.thr);
      me1 = me + a.tau * (ve - cxe);
      ne1 = ne + a.tau * (xe - ze);
    };
    float2 v1, z1, m1, n1;
    upd(x.x, cx.x, m0.x, n0.x, py.x, om.x, v1.x, z1.x, m1.x, n1.x);
    upd(x.y, cx.y, m0.y, n0.y, py.y, om.y, v1.y, z1.y, m1.y, n1.y);
    if constexpr (LAST) {
      const size_t j = (size_t)i * N2 + j2_0 + c;
      reinterpret_cast<float2*>(a.x)[j] = x;
      reinterpret_cast<float2*>(a.v)[j] = v1;
      reinterpret_cast<float2*>(a.z)[j] = z1;
      reinterpret_cast<float2*>(a.mu)[j] = m1;
      reinterpret_cast<float2*>(a.nu)[j] = n1;
    } else {
      a.mu_b[qb] = m1;
      a.nu_b[qb] = n1;
      lds[lp(i * S + c)] = cadd(v1, m1);        // a = v + mu
      lds[lp(i * S + CB + c)] = csub(z1, n1);   // b = z - nu
    }
  }
  if constexpr (!LAST) {
    __syncthreads();
    lds_fft<N1, S, T, false, true, N1>(lds, tws, tid);
#pragma unroll 1
    for (int k0 = 0; k0 < EPT; k0 += CH) {
      float2 t[CH];
      int l[CH];
      size_t go[CH];
#pragma unroll
      for (int k = 0; k < CH; ++k) {
        const int e = tid + (k0 + k) * T;
        if (FULL || e < NE) {
          int ex;
          gaddr(e, go[k], l[k], ex);
          t[k] = cp_twN(a, ex);
        }
      }
#pragma unroll
      for (int k = 0; k < CH; ++k) {
        const int e = tid + (k0 + k) * T;
        if (FULL || e < NE) a.Yab[go[k]] = cmul(lds[lp(l[k])], t[k]);
      }
    }
  }
}

// Columns per column-pass workgroup: 4 when N1 >= 512 (two signals' columns
// then fill 64 KiB of LDS), else 8.
constexpr int cp_cb(int N1) { return N1 >= 512 ? 4 : 8; }
// Column-pass threads: 512 from N1 = 512 on (16 values per thread), else 256.
constexpr int cp_col_threads(int N1) { return N1 >= 512 ? 512 : 256; }
// Largest row / column lengths of these passes (n <= 2^22).
constexpr int kCpMaxN2 = 2048;
constexpr int kCpMaxN1 = 1024;

}  // namespace cs
