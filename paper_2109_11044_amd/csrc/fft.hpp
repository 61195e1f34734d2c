// fft.hpp -- LDS-resident Stockham FFT building blocks for gfx950.
//
// A workgroup transforms `nb` independent sequences of length T held in LDS.
// Element e of sequence b sits at lds[b * bs + e * es] (rows: es = 1,
// bs = T; column panels: es = nb, bs = 1).  Each radix-R stage reads all of
// a thread's butterflies into registers, synchronises, and writes the
// results (so one buffer suffices), with the Stockham autosort indexing:
//   butterfly j in [0, T/R), k = j mod Ns (Ns = product of earlier radices)
//   in : x_q = a[j + q T/R] * W_T^(k q T/(Ns R))
//   out: a[(j / Ns) Ns R + k + q Ns] = DFT_R(x)_q
// Twiddles come from a table tw[t] = exp(-2 pi i t / T) (conjugated for the
// inverse transform).  Forward transforms use exp(-2 pi i jk/T); neither
// direction is scaled.
#pragma once

#include <hip/hip_runtime.h>

namespace cesim {

template <typename real> struct cpx_t;
template <> struct cpx_t<float> { using type = float2; };
template <> struct cpx_t<double> { using type = double2; };
template <typename real> using cpx = typename cpx_t<real>::type;

template <typename C> __device__ __forceinline__ C cadd(C a, C b) { return {a.x + b.x, a.y + b.y}; }
template <typename C> __device__ __forceinline__ C csub(C a, C b) { return {a.x - b.x, a.y - b.y}; }
template <typename C> __device__ __forceinline__ C cmul(C a, C b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename C> __device__ __forceinline__ C cmulconj(C a, C b) {   // a * conj(b)
  return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
// multiply by -i (forward) or +i (inverse)
template <bool INV, typename C> __device__ __forceinline__ C rot90(C a) {
  return INV ? C{-a.y, a.x} : C{a.y, -a.x};
}
template <typename C, typename R> __device__ __forceinline__ C cscale(C a, R s) { return {a.x * s, a.y * s}; }

constexpr double kC5a = 0.3090169943749474241;    // cos(2 pi / 5)
constexpr double kC5b = -0.8090169943749474241;   // cos(4 pi / 5)
constexpr double kS5a = 0.95105651629515357212;   // sin(2 pi / 5)
constexpr double kS5b = 0.58778525229247312917;   // sin(4 pi / 5)
constexpr double kS3 = 0.86602540378443864676;    // sin(2 pi / 3)
constexpr double kR2 = 0.7071067811865475244;     // 1 / sqrt(2)

// In-register DFT of radix R (unscaled); forward sign exp(-2 pi i/R).
template <int R, bool INV, typename real>
__device__ __forceinline__ void dft(cpx<real>* x) {
  using C = cpx<real>;
  if constexpr (R == 2) {
    const C a = x[0], b = x[1];
    x[0] = cadd(a, b);
    x[1] = csub(a, b);
  } else if constexpr (R == 4) {
    const C t0 = cadd(x[0], x[2]), t1 = csub(x[0], x[2]);
    const C t2 = cadd(x[1], x[3]), t3 = rot90<INV>(csub(x[1], x[3]));
    x[0] = cadd(t0, t2);
    x[2] = csub(t0, t2);
    x[1] = cadd(t1, t3);
    x[3] = csub(t1, t3);
  } else if constexpr (R == 8) {
    C e[4] = {x[0], x[2], x[4], x[6]};
    C o[4] = {x[1], x[3], x[5], x[7]};
    dft<4, INV, real>(e);
    dft<4, INV, real>(o);
    const real r2 = (real)kR2;
    // o_k *= W8^k
    o[1] = INV ? C{(o[1].x - o[1].y) * r2, (o[1].x + o[1].y) * r2}
               : C{(o[1].x + o[1].y) * r2, (o[1].y - o[1].x) * r2};
    o[2] = rot90<INV>(o[2]);
    o[3] = INV ? C{-(o[3].x + o[3].y) * r2, (o[3].x - o[3].y) * r2}
               : C{(o[3].y - o[3].x) * r2, -(o[3].x + o[3].y) * r2};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      x[k] = cadd(e[k], o[k]);
      x[k + 4] = csub(e[k], o[k]);
    }
  } else if constexpr (R == 3) {
    const C t = cadd(x[1], x[2]);
    const C m = {x[0].x - (real)0.5 * t.x, x[0].y - (real)0.5 * t.y};
    const C d = cscale(rot90<INV>(csub(x[1], x[2])), (real)kS3);
    x[0] = cadd(x[0], t);
    x[1] = cadd(m, d);
    x[2] = csub(m, d);
  } else if constexpr (R == 5) {
    const C a1 = cadd(x[1], x[4]), a2 = cadd(x[2], x[3]);
    const C b1 = csub(x[1], x[4]), b2 = csub(x[2], x[3]);
    const real c1 = (real)kC5a, c2 = (real)kC5b, s1 = (real)kS5a, s2 = (real)kS5b;
    const C r1 = {x[0].x + c1 * a1.x + c2 * a2.x, x[0].y + c1 * a1.y + c2 * a2.y};
    const C r2 = {x[0].x + c2 * a1.x + c1 * a2.x, x[0].y + c2 * a1.y + c1 * a2.y};
    const C i1 = rot90<INV>(C{s1 * b1.x + s2 * b2.x, s1 * b1.y + s2 * b2.y});
    const C i2 = rot90<INV>(C{s2 * b1.x - s1 * b2.x, s2 * b1.y - s1 * b2.y});
    x[0] = cadd(x[0], cadd(a1, a2));
    x[1] = cadd(r1, i1);
    x[4] = csub(r1, i1);
    x[2] = cadd(r2, i2);
    x[3] = csub(r2, i2);
  }
}

// Radix plan: T = product of rad[0..nst).
struct Plan {
  int T;
  int nst;
  int rad[16];
};

// One Stockham stage over all nb sequences.  NTHR threads, each handling up
// to ceil(E / R) butterflies (E = elements per thread the kernel was built
// for).  BFAST: butterfly index maps sequence-fastest (column panels).
template <int R, bool INV, int NTHR, int E, bool BFAST, typename real>
__device__ __forceinline__ void stockham_stage(cpx<real>* lds, int T, int Ns, int nb, int es,
                                               int bs, const cpx<real>* __restrict__ tw) {
  using C = cpx<real>;
  constexpr int NBF = (E + R - 1) / R;
  const int nbt = T / R;
  const int total = nb * nbt;
  const int tstep = T / (Ns * R);
  C x[NBF][R];
  int obase[NBF];
#pragma unroll
  for (int i = 0; i < NBF; ++i) {
    const int f = threadIdx.x + i * NTHR;
    obase[i] = -1;
    if (f < total) {
      const int b = BFAST ? f % nb : f / nbt;
      const int j = BFAST ? f / nb : f % nbt;
      const int k = j % Ns;
      const C* src = lds + b * bs;
#pragma unroll
      for (int q = 0; q < R; ++q) x[i][q] = src[(j + q * nbt) * es];
      if (Ns > 1) {
#pragma unroll
        for (int q = 1; q < R; ++q) {
          const C w = tw[k * q * tstep];
          x[i][q] = INV ? cmulconj(x[i][q], w) : cmul(x[i][q], w);
        }
      }
      dft<R, INV, real>(x[i]);
      obase[i] = b * bs + ((j / Ns) * Ns * R + k) * es;
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NBF; ++i) {
    if (obase[i] >= 0) {
#pragma unroll
      for (int q = 0; q < R; ++q) lds[obase[i] + q * Ns * es] = x[i][q];
    }
  }
  __syncthreads();
}

// Full transform: all stages of the plan.  Expects the data in LDS and a
// barrier before the call; leaves the result in LDS after a barrier.
template <bool INV, int NTHR, int E, bool BFAST, typename real>
__device__ void fft_lds(cpx<real>* lds, const Plan& p, int nb, int es, int bs,
                        const cpx<real>* __restrict__ tw) {
  int Ns = 1;
  for (int s = 0; s < p.nst; ++s) {
    const int R = p.rad[s];
    switch (R) {
      case 8: stockham_stage<8, INV, NTHR, E, BFAST, real>(lds, p.T, Ns, nb, es, bs, tw); break;
      case 4: stockham_stage<4, INV, NTHR, E, BFAST, real>(lds, p.T, Ns, nb, es, bs, tw); break;
      case 2: stockham_stage<2, INV, NTHR, E, BFAST, real>(lds, p.T, Ns, nb, es, bs, tw); break;
      case 3: stockham_stage<3, INV, NTHR, E, BFAST, real>(lds, p.T, Ns, nb, es, bs, tw); break;
      default: stockham_stage<5, INV, NTHR, E, BFAST, real>(lds, p.T, Ns, nb, es, bs, tw); break;
    }
    Ns *= R;
  }
}

}  // namespace cesim
