// fft_pow2.hpp -- register-resident Stockham FFT for lengths T = 2^a or
// T = 3 * 2^a known at compile time (the draw's hot path).
//
// Each thread owns E elements of one transform (E = 16, or 24 when 3 | T),
// its "home" positions base + S h (h < E, S = T / E threads per
// transform).  A stage of radix R (R | E) treats them as U = E / R
// butterflies j = base + S u with inputs h = u + q U (positions j + q T / R),
// applies the Stockham twiddles and an in-register radix-R DFT.  Its outputs
// belong at positions (j / Ns) Ns R + (j mod Ns) + q Ns; unless the stage is
// the last one (whose outputs land on the home positions), they are
// exchanged through LDS and every thread reloads its home positions.
// Forward plans are [16, ..., 16, r] for 2^a and [8, ..., 8, r, 3] for
// 3 * 2^a, inverse plans the reverse (r = the remaining power of two), so a forward
// transform followed by an inverse one needs no exchange in between:
// pointwise scaling happens in registers.
// Twiddles: w1 = table[k T / (Ns R)] from exp(-2 pi i t / T), higher powers
// by binary powering (each a product of at most four rounded factors).
#pragma once

#include "fft.hpp"

namespace cesim {

constexpr int ilog2c(int x) { return x <= 1 ? 0 : 1 + ilog2c(x / 2); }

// Elements per thread for length T.
template <int T>
constexpr int p2_elems() { return T % 3 == 0 ? 24 : 16; }

template <int T, bool INV>
struct P2Plan {
  static constexpr bool THREE = T % 3 == 0;
  static constexpr int LB = THREE ? 3 : 4;           // log2 of the main radix (8 or 16)
  static constexpr int L = ilog2c(THREE ? T / 3 : T);
  static constexpr int REM = L % LB;
  static constexpr int NMAIN = L / LB;
  static constexpr int NST = NMAIN + (REM ? 1 : 0) + (THREE ? 1 : 0);
  static constexpr int fwd_radix(int s) {
    return s < NMAIN ? (1 << LB) : ((s == NMAIN && REM) ? (1 << REM) : 3);
  }
  static constexpr int radix(int s) { return INV ? fwd_radix(NST - 1 - s) : fwd_radix(s); }
  static constexpr int ns(int s) {
    int n = 1;
    for (int i = 0; i < s; ++i) n *= radix(i);
    return n;
  }
};

// W16^m, m in {1, 2, 3, 6, 9} for the forward sign (conjugated for INV).
template <bool INV, typename real>
__device__ __forceinline__ cpx<real> w16(int m) {
  constexpr double c1 = 0.92387953251128675613, s1 = 0.38268343236508977173;
  double re, im;
  switch (m) {
    case 1: re = c1; im = -s1; break;
    case 2: re = kR2; im = -kR2; break;
    case 3: re = s1; im = -c1; break;
    case 6: re = -kR2; im = -kR2; break;
    default: re = -c1; im = s1; break;    // 9
  }
  return {(real)re, (real)(INV ? -im : im)};
}

// In-register radix-16 DFT as 4 x 4: x_{i + 4r} -> X_{s + 4t}.
template <bool INV, typename real>
__device__ __forceinline__ void dft16(cpx<real>* x) {
  using C = cpx<real>;
  C y[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    C t[4] = {x[i], x[i + 4], x[i + 8], x[i + 12]};
    dft<4, INV, real>(t);
#pragma unroll
    for (int s = 0; s < 4; ++s) y[i][s] = t[s];
  }
  // twiddles W16^(i s)
  y[1][1] = cmul(y[1][1], w16<INV, real>(1));
  y[1][2] = cmul(y[1][2], w16<INV, real>(2));
  y[1][3] = cmul(y[1][3], w16<INV, real>(3));
  y[2][1] = cmul(y[2][1], w16<INV, real>(2));
  y[2][2] = rot90<INV>(y[2][2]);                  // W16^4
  y[2][3] = cmul(y[2][3], w16<INV, real>(6));
  y[3][1] = cmul(y[3][1], w16<INV, real>(3));
  y[3][2] = cmul(y[3][2], w16<INV, real>(6));
  y[3][3] = cmul(y[3][3], w16<INV, real>(9));
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    C t[4] = {y[0][s], y[1][s], y[2][s], y[3][s]};
    dft<4, INV, real>(t);
#pragma unroll
    for (int tt = 0; tt < 4; ++tt) x[s + 4 * tt] = t[tt];
  }
}

template <int R, bool INV, typename real>
__device__ __forceinline__ void dft_any(cpx<real>* x) {
  if constexpr (R == 16) dft16<INV, real>(x);
  else dft<R, INV, real>(x);
}

// Powers w^1 .. w^(R-1) of w by binary powering.
template <int R, typename C>
__device__ __forceinline__ void powers(C w1, C* w) {
  w[1] = w1;
#pragma unroll
  for (int q = 2; q < R; ++q) {
    const int hb = 1 << (31 - __builtin_clz(q));
    w[q] = (hb == q) ? cmul(w[q / 2], w[q / 2]) : cmul(w[hb], w[q - hb]);
  }
}

// LDS layouts: one padding element per 16 positions.
template <typename C>
struct RowLds {
  C* p;
  __device__ __forceinline__ C load(int pos) const { return p[pos + (pos >> 4)]; }
  __device__ __forceinline__ void store(int pos, C v) const { p[pos + (pos >> 4)] = v; }
};
template <typename C>
struct ColLds {              // 2^lcp interleaved columns
  C* p;
  int c, lcp;
  __device__ __forceinline__ C load(int pos) const { return p[((pos + (pos >> 4)) << lcp) + c]; }
  __device__ __forceinline__ void store(int pos, C v) const {
    p[((pos + (pos >> 4)) << lcp) + c] = v;
  }
};

template <typename real, int T, bool INV, int s, typename Lds>
__device__ __forceinline__ void p2_stages(cpx<real> (&x)[p2_elems<T>()], int base,
                                          const cpx<real>* __restrict__ tw, const Lds& lds) {
  using PL = P2Plan<T, INV>;
  using C = cpx<real>;
  constexpr int E = p2_elems<T>();
  if constexpr (s < PL::NST) {
    constexpr int R = PL::radix(s), Ns = PL::ns(s), S = T / E, U = E / R;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int j = base + S * u;
      C v[R];
#pragma unroll
      for (int q = 0; q < R; ++q) v[q] = x[u + q * U];
      if constexpr (Ns > 1) {
        const int k = j % Ns;
        C w[R];
        powers<R>(tw[k * (T / (Ns * R))], w);
#pragma unroll
        for (int q = 1; q < R; ++q) v[q] = INV ? cmulconj(v[q], w[q]) : cmul(v[q], w[q]);
      }
      dft_any<R, INV, real>(v);
#pragma unroll
      for (int q = 0; q < R; ++q) x[u + q * U] = v[q];
    }
    if constexpr (s + 1 < PL::NST) {
      __syncthreads();
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int j = base + S * u;
        const int ob = (j / Ns) * Ns * R + j % Ns;
#pragma unroll
        for (int q = 0; q < R; ++q) lds.store(ob + q * Ns, x[u + q * U]);
      }
      __syncthreads();
#pragma unroll
      for (int h = 0; h < E; ++h) x[h] = lds.load(base + S * h);
      p2_stages<real, T, INV, s + 1>(x, base, tw, lds);
    }
  }
}

// Whole transform on the home layout (input and output on home positions).
template <typename real, int T, bool INV, typename Lds>
__device__ __forceinline__ void p2_fft(cpx<real> (&x)[p2_elems<T>()], int base,
                                       const cpx<real>* __restrict__ tw, const Lds& lds) {
  p2_stages<real, T, INV, 0>(x, base, tw, lds);
}

// Largest launch shapes of the register-FFT kernels (the kernels take any
// power-of-two number of rows or columns per workgroup up to these).
template <int T>
struct P2Rows {
  static constexpr int E = p2_elems<T>();
  static constexpr int S = T / E;                     // threads per row
  static constexpr int ROWS = S >= 256 ? 1 : 256 / S;  // rows per workgroup
  static constexpr int NTHR = ROWS * S;
  static constexpr int LD = T + T / 16;               // padded row length
};

template <typename real, int T>
struct P2Cols {
  static constexpr int E = p2_elems<T>();
  static constexpr int S = T / E;
  static constexpr int LD = T + T / 16;
  static constexpr int cap_thr = 1024 / S;
  static constexpr int cap_lds = (int)((160 * 1024) / (LD * sizeof(cpx<real>)));
  static constexpr int cmin(int a, int b) { return a < b ? a : b; }
  static constexpr int pow2floor(int v) { int p = 1; while (p * 2 <= v) p *= 2; return p; }
  static constexpr int CP = pow2floor(cmin(16, cmin(cap_thr, cap_lds)));
  static constexpr int NTHR = CP * S;
};

}  // namespace cesim
