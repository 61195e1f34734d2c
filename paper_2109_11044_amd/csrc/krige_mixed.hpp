// krige_mixed.hpp -- device code of the mixed-precision grid product
// (step 5 of Section 2, eq. (4) of Section 3) shared by the translation
// units that instantiate it: krige.hip (the tiles of two node fragments per
// wave and the 8-wave tile) and krige_tile1.hip (the tiles of one node
// fragment per wave, built with machine sinking off so that the coefficient
// reads stay ahead of the conditional matrix instructions).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.hpp"

namespace cesim {

typedef double doublex4 __attribute__((ext_vector_type(4)));
typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4v __attribute__((ext_vector_type(4)));   // 16 bytes, register-promotable
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

// Half-precision element types of the split product: the vector type and
// the matching 32x32x16 matrix-core instruction.
template <typename H> struct HalfOps;
template <> struct HalfOps<__bf16> {
  using V = bf16x8;
  static constexpr bool kF16 = false;
  static __device__ __forceinline__ floatx16 mfma(V a, V b, floatx16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
  }
};
template <> struct HalfOps<_Float16> {
  using V = f16x8;
  static constexpr bool kF16 = true;
  static __device__ __forceinline__ floatx16 mfma(V a, V b, floatx16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
  }
};

constexpr int kKC = kGemmChunk;   // observations per k-chunk of the mixed kernel

// Grid GEMM, mixed precision.  The product is formed transposed,
// D[r][g] = sum_i B[r][i] K12[g][i], so that the accumulator's lane index
// runs over grid nodes and every store writes runs of 32 consecutive nodes.
// Workgroup: 4 waves, 128 NF grid nodes x 256 realizations; wave w owns
// nodes [32 NF w, 32 NF (w + 1)) as NF 32-node fragments and all 8 blocks of
// 32 realizations (8 NF accumulators).  Coefficient chunks of 32
// observations are double-buffered in LDS: the next chunk is fetched into
// registers while the current one is multiplied, and each coefficient
// fragment read from LDS feeds all NF node fragments.  Per chunk each lane
// evaluates 16 NF correlations (NF nodes x 16 observations) in FP32 and splits
// them into bf16 hi/lo; 3 products hi.hi + lo.hi + hi.lo per block.
// Layout of v_mfma_f32_32x32x16_bf16: lane l holds A[l % 32][8 (l/32) + j]
// and B[8 (l/32) + j][l % 32]; accumulator e of lane l is
// D[8 (e/4) + 4 (l/32) + e % 4][l % 32].
// One correlation in FP32 (scaled by ks) and its half-precision hi / lo
// split; every split kernel evaluates correlations through this function.
template <int NU>
__device__ __forceinline__ float corr_f32(float gxt, float gyt, float2 s) {
  const float hx = gxt - s.x, hy = gyt - s.y;
  return rho_scaled_f32(NU, __builtin_amdgcn_sqrtf(hx * hx + hy * hy));
}

template <int NU, typename H>
__device__ __forceinline__ void corr_split(float gxt, float gyt, float2 s, float ks, H& h, H& l) {
  const float c = ks * corr_f32<NU>(gxt, gyt, s);
  h = (H)c;
  l = (H)(c - (float)h);
}

// The FP16 split of two correlations e0, e1 (times ks, a power of two, so
// that ks e is exact in FP32) into one register of hi halves and one of lo
// halves: hi = half(ks e) and lo = half(ks e - hi), each by one fused
// multiply-add rounded once to FP16 into the low or high half -- the values
// of corr_split, in two instructions per correlation where the compiler's
// own code (a multiply and a packed conversion for hi, then hi once more to
// feed lo) takes three and a half.
__device__ __forceinline__ void split_pair_f16(float ks, float e0, float e1, uint32_t& h,
                                               uint32_t& l) {
  asm("v_fma_mixlo_f16 %0, %1, %2, 0\n\t"
      "v_fma_mixhi_f16 %0, %1, %3, 0"
      : "=&v"(h)
      : "v"(ks), "v"(e0), "v"(e1));
  asm("v_fma_mixlo_f16 %0, %1, %2, -%3 op_sel_hi:[0,0,1]\n\t"
      "v_fma_mixhi_f16 %0, %1, %4, -%3 op_sel:[0,0,1] op_sel_hi:[0,0,1]"
      : "=&v"(l)
      : "v"(ks), "v"(e0), "v"(h), "v"(e1));
}

// Grid coordinates of node g in range units (the map U, scaled per path).
__device__ __forceinline__ void node_coords(int g, int m1, float dx, float dy, float ux, float uxy,
                                            float uyx, float uy, float& gxt, float& gyt) {
  const float gx = (float)(g % m1) * dx, gy = (float)(g / m1) * dy;
  gxt = ux * gx + uxy * gy;
  gyt = uyx * gx + uy * gy;
}

// Bounding circle, in scaled coordinates, of the grid nodes g0 .. g0 + TG - 1
// (flattened, x fastest): the rectangle of their rows and columns mapped by U.
__device__ __forceinline__ void tile_circle(int g0, int TG, int M, int m1, float dx, float dy,
                                            float ux, float uxy, float uyx, float uy, float& cx,
                                            float& cy, float& rad) {
  const int ga = g0, gb = min(g0 + TG, M) - 1;
  const int ja = ga / m1, jb = gb / m1;
  const int ia = ja == jb ? ga % m1 : 0, ib = ja == jb ? gb % m1 : m1 - 1;
  const float x = 0.5f * (float)(ia + ib) * dx, y = 0.5f * (float)(ja + jb) * dy;
  const float hx = 0.5f * (float)(ib - ia) * dx, hy = 0.5f * (float)(jb - ja) * dy;
  cx = ux * x + uxy * y;
  cy = uyx * x + uy * y;
  const float ax = ux * hx + uxy * hy, ay = uyx * hx + uy * hy;   // half-diagonals
  const float bx = ux * hx - uxy * hy, by = uyx * hx - uy * hy;
  rad = __builtin_amdgcn_sqrtf(fmaxf(ax * ax + ay * ay, bx * bx + by * by)) * 1.0001f + 1e-3f;
}

template <int NU, typename H>
__device__ __forceinline__ void k12_frag(float gxt, float gyt, const float2* __restrict__ sv,
                                         float ks, typename HalfOps<H>::V& ah,
                                         typename HalfOps<H>::V& al) {
  if constexpr (HalfOps<H>::kF16) {
    u32x4v hw, lw;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      uint32_t h, l;
      split_pair_f16(ks, corr_f32<NU>(gxt, gyt, sv[2 * q]), corr_f32<NU>(gxt, gyt, sv[2 * q + 1]),
                     h, l);
      hw[q] = h;
      lw[q] = l;
    }
    ah = __builtin_bit_cast(typename HalfOps<H>::V, hw);
    al = __builtin_bit_cast(typename HalfOps<H>::V, lw);
  } else {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      H h, l;
      corr_split<NU, H>(gxt, gyt, sv[j], ks, h, l);
      ah[j] = h;
      al[j] = l;
    }
  }
}

// Correlations of one k-step for the lanes of a wave: lane l holds
// observations sv[8 (l / 32) + j], j < 8, for its NF nodes (FP32, split into
// half-precision hi / lo; correlations scaled by ks).
template <int NU, int NF, typename H>
__device__ __forceinline__ void k12_step(const float2* sv, bool upper, const float (&gxt)[NF],
                                         const float (&gyt)[NF], float ks,
                                         typename HalfOps<H>::V (&ah)[NF],
                                         typename HalfOps<H>::V (&al)[NF]) {
  const float2* p = sv + (upper ? 8 : 0);
  if constexpr (HalfOps<H>::kF16) {
    u32x4v hw[NF], lw[NF];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const float2 s0 = p[2 * q], s1 = p[2 * q + 1];
#pragma unroll
      for (int f = 0; f < NF; ++f) {
        uint32_t h, l;
        split_pair_f16(ks, corr_f32<NU>(gxt[f], gyt[f], s0), corr_f32<NU>(gxt[f], gyt[f], s1), h,
                       l);
        hw[f][q] = h;
        lw[f][q] = l;
      }
    }
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      ah[f] = __builtin_bit_cast(typename HalfOps<H>::V, hw[f]);
      al[f] = __builtin_bit_cast(typename HalfOps<H>::V, lw[f]);
    }
  } else {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const float2 sj = p[j];
#pragma unroll
      for (int f = 0; f < NF; ++f) {
        H h, l;
        corr_split<NU, H>(gxt[f], gyt[f], sj, ks, h, l);
        ah[f][j] = h;
        al[f][j] = l;
      }
    }
  }
}

// Whether any lane of the wave holds a half with a nonzero bit pattern in
// v (uniform).  A fragment of exact zeros multiplies to exact zeros, so its
// products are skipped without changing a bit of the sums: the low halves
// of the FP16 split vanish once ks C falls into FP16's subnormal range (the
// high half then holds the whole value), and both halves of correlations
// below half the smallest subnormal.
template <typename HV>
__device__ __forceinline__ bool wave_any_nonzero(const HV& v) {
  const u32x4v w = __builtin_bit_cast(u32x4v, v);
  return __builtin_amdgcn_ballot_w64((w[0] | w[1] | w[2] | w[3]) != 0u) != 0;
}

// Three products hi.hi + hi.lo + lo.hi of one k-step (ks = 0 or 16 within
// the chunk) for the 8 blocks of 32 realizations whose coefficients start at
// sh / sl (rows of 32 observations, swizzled as stored).
template <int NF, typename H>
__device__ __forceinline__ void mfma_step(const H* __restrict__ sh, const H* __restrict__ sl,
                                          int ks, int lane, const typename HalfOps<H>::V (&ah)[NF],
                                          const typename HalfOps<H>::V (&al)[NF],
                                          floatx16 (&acc)[NF][8]) {
  using HV = typename HalfOps<H>::V;
  const int kb = (lane >> 5) * 8;
  bool nzh[NF], nzl[NF];
#pragma unroll
  for (int f = 0; f < NF; ++f) {
    nzh[f] = wave_any_nonzero(ah[f]);
    nzl[f] = wave_any_nonzero(al[f]);
  }
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    const int rr = 32 * b + (lane & 31);
    const int pc = ((ks + kb) >> 3) ^ ((rr >> 2) & 3);
    const HV bh = *reinterpret_cast<const HV*>(&sh[rr * kKC + 8 * pc]);
    const HV bl = *reinterpret_cast<const HV*>(&sl[rr * kKC + 8 * pc]);
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      if (nzh[f]) acc[f][b] = HalfOps<H>::mfma(bh, ah[f], acc[f][b]);
      if (nzl[f]) acc[f][b] = HalfOps<H>::mfma(bh, al[f], acc[f][b]);
      if (nzh[f]) acc[f][b] = HalfOps<H>::mfma(bl, ah[f], acc[f][b]);
    }
  }
}

template <int NU, int NF, int NB, typename H>
__global__ void __launch_bounds__(256, NF * NB > 8 ? 1 : 2)
k_krige_split3(float* __restrict__ fields, int m1, int M, int R, int Rp,
               const H* __restrict__ Bh, const H* __restrict__ Bl,
               const float* __restrict__ colscale, const float* __restrict__ yhat, int n,
               const float2* __restrict__ st, const float4* __restrict__ circ, float xcut,
               float ux, float uxy, float uyx, float uy, float dx, float dy, float kscale,
               const int* __restrict__ fail) {
  if (fail[0] & 2) return;   // failed factorisation: the fields stay as drawn
  using HV = typename HalfOps<H>::V;
  constexpr int TG = 128 * NF, TR = 32 * NB;
  constexpr int NQ = TR * kKC / 8 / 256;      // 16-byte pieces per thread and chunk
  __shared__ __align__(16) H Sh[2][TR * kKC];
  __shared__ __align__(16) H Sl[2][TR * kKC];
  __shared__ float2 Ss[2][kKC];
  const int g0 = blockIdx.x * TG, r0 = blockIdx.y * TR;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  float gxt[NF], gyt[NF];
#pragma unroll
  for (int f = 0; f < NF; ++f)
    node_coords(min(g0 + 32 * NF * wave + 32 * f + (lane & 31), M - 1), m1, dx, dy, ux, uxy,
                uyx, uy, gxt[f], gyt[f]);
  const int kb = (lane >> 5) * 8;
  floatx16 acc[NF][NB];
#pragma unroll
  for (int f = 0; f < NF; ++f)
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[f][b][e] = 0.0f;
  const int nchunks = (n + kKC - 1) / kKC;
  u32x4v ph[NQ], pl[NQ];
  float2 ps = {0.f, 0.f};
  auto fetch = [&](int kc) {
    const u32x4v* gh = reinterpret_cast<const u32x4v*>(Bh + ((size_t)kc * Rp + r0) * kKC);
    const u32x4v* gl = reinterpret_cast<const u32x4v*>(Bl + ((size_t)kc * Rp + r0) * kKC);
#pragma unroll
    for (int u = 0; u < NQ; ++u) {
      ph[u] = gh[threadIdx.x + 256 * u];
      pl[u] = gl[threadIdx.x + 256 * u];
    }
    if (threadIdx.x < kKC) ps = st[min(kc * kKC + (int)threadIdx.x, n - 1)];
  };
  // LDS rows of 4 x 16 B; the 16-byte column is XOR-swizzled by bits 2-3
  // of the row so that 16 consecutive rows read at one column hit 16
  // distinct bank groups.
  auto stash = [&](int buf) {
    u32x4v* sh = reinterpret_cast<u32x4v*>(Sh[buf]);
    u32x4v* sl = reinterpret_cast<u32x4v*>(Sl[buf]);
#pragma unroll
    for (int u = 0; u < NQ; ++u) {
      const int q = threadIdx.x + 256 * u, row = q >> 2;
      const int pq = (row << 2) | ((q & 3) ^ ((row >> 2) & 3));
      sh[pq] = ph[u];
      sl[pq] = pl[u];
    }
    if (threadIdx.x < kKC) Ss[buf][threadIdx.x] = ps;
  };
  // Chunks whose every correlation with this tile's nodes rounds to zero in
  // the half-precision split are skipped: their products would add exact
  // zeros.  The test (uniform over the workgroup) compares the distance of
  // the tile's bounding circle to the chunk's with the cut-off distance.
  float tcx, tcy, trad;
  tile_circle(g0, TG, M, m1, dx, dy, ux, uxy, uyx, uy, tcx, tcy, trad);
  // The test runs for 64 chunks at once, one per lane, into a wave-wide
  // mask (the same in every wave of the workgroup), so that finding the
  // next live chunk waits for one load per 64 chunks, not one per chunk.
  uint64_t mask = 0;
  int base = -64;
  auto next_live = [&](int kc) {
    for (;;) {
      if (kc >= nchunks) return nchunks;
      if (kc >= base + 64) {
        base = kc;
        const int q = base + lane;
        bool lv = false;
        if (q < nchunks) {
          const float4 c4 = circ[q];
          const float ddx = tcx - c4.x, ddy = tcy - c4.y;
          lv = __builtin_amdgcn_sqrtf(ddx * ddx + ddy * ddy) - trad - c4.z < xcut;
        }
        mask = __builtin_amdgcn_ballot_w64(lv);
      }
      const uint64_t m = mask >> (kc - base);
      if (m) return kc + (int)__builtin_ctzll(m);
      kc = base + 64;
    }
  };
  int kc = next_live(0);
  if (kc < nchunks) {
    fetch(kc);
    stash(0);
  }
  __syncthreads();
  for (int buf = 0; kc < nchunks; buf ^= 1) {
    const int kn = next_live(kc + 1);
    if (kn < nchunks) fetch(kn);
#pragma unroll
    for (int ks = 0; ks < kKC; ks += 16) {
      float2 sv[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) sv[j] = Ss[buf][ks + kb + j];
      HV ah[NF], al[NF];
      bool nzh[NF], nzl[NF];
#pragma unroll
      for (int f = 0; f < NF; ++f) {
        k12_frag<NU, H>(gxt[f], gyt[f], sv, kscale, ah[f], al[f]);
        // tiles of 64 and 128 realizations issue too few products per
        // fragment for the test and its branches to pay
        nzh[f] = NB < 8 || wave_any_nonzero(ah[f]);
        nzl[f] = NB < 8 || wave_any_nonzero(al[f]);
      }
      // Coefficient fragments of block b; with one node fragment per wave
      // they are read a block ahead, before the (conditional) products of
      // the block before.  (Machine sinking, off where these tiles are
      // built, would move such reads back below those branches.)
      auto coef = [&](int b, HV& h, HV& l) {
        const int rr = 32 * b + (lane & 31);
        const int pc = ((ks + kb) >> 3) ^ ((rr >> 2) & 3);
        h = *reinterpret_cast<const HV*>(&Sh[buf][rr * kKC + 8 * pc]);
        l = *reinterpret_cast<const HV*>(&Sl[buf][rr * kKC + 8 * pc]);
      };
      constexpr int kAhead = NF == 1 ? 1 : 0, kBuf = kAhead + 1;
      HV bh[kBuf], bl[kBuf];
#pragma unroll
      for (int b = 0; b < kAhead; ++b) coef(b, bh[b], bl[b]);
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        if (b + kAhead < NB) coef(b + kAhead, bh[(b + kAhead) % kBuf], bl[(b + kAhead) % kBuf]);
        const int u = b % kBuf;
#pragma unroll
        for (int f = 0; f < NF; ++f) {
          if (nzh[f]) acc[f][b] = HalfOps<H>::mfma(bh[u], ah[f], acc[f][b]);
          if (nzl[f]) acc[f][b] = HalfOps<H>::mfma(bh[u], al[f], acc[f][b]);
          if (nzh[f]) acc[f][b] = HalfOps<H>::mfma(bl[u], ah[f], acc[f][b]);
        }
      }
    }
    if (kn < nchunks) stash(buf ^ 1);
    __syncthreads();
    kc = kn;
  }
#pragma unroll
  for (int f = 0; f < NF; ++f) {
    const int gg = g0 + 32 * NF * wave + 32 * f + (lane & 31);
    if (gg >= M) continue;
    const float yh = yhat[gg];
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int r = r0 + 32 * b + 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3);
        if (r < R) fields[(size_t)r * M + gg] += fmaf(acc[f][b][e], colscale[r], yh);
      }
  }
}

// Launches k_krige_split3<nu, 1, nb, H> (one node fragment per wave; nb =
// 2, 4 or 8 blocks of 32 realizations; H = FP16 when f16, else BF16) on
// stream s with the kernel's arguments; defined in krige_tile1.hip.
cesim_status launch_split3_one_fragment(int nu, int nb, bool f16, dim3 grid, hipStream_t s,
                                        float* fields, int m1, int M, int R, int Rp,
                                        const void* Bh, const void* Bl, const float* colscale,
                                        const float* yhat, int n, const float2* st,
                                        const float4* circ, float xcut, float ux, float uxy,
                                        float uyx, float uy, float dx, float dy, float kscale,
                                        const int* fail);

}  // namespace cesim
