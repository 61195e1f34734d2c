// krige.hip -- Kriging of the residual coefficients onto the grid (step 5 of
// Section 2; the grid prediction of eq. (4), Section 3):
//   v_r[g] = y_r[g] + sum_i C(g - s_i) B[r][i],
// a dense contraction over the observations whose left factor K12 is far too
// large to store (M x n), so every workgroup generates its K12 tile in
// registers, directly in the matrix-core operand layout, from transformed
// coordinates: x = |U g - U s| is the lag length in range units.
//
//   FP64 path : v_mfma_f64_16x16x4f64, K12 and B in FP64.
//   mixed path: K12 in FP32, split into half-precision hi + lo; B scaled per
//               realization into [-1, 1] and split likewise; three 32x32x16
//               matrix-core products hi.hi + hi.lo + lo.hi accumulate in FP32.
//               The half type is FP16 (11-bit significands: the split keeps
//               about 22 bits, and K12 is scaled by 2^12 so that small
//               correlations stay normal) or BF16 (8-bit significands: about
//               16 bits); both run at the same matrix-core rate.
#include <hip/hip_runtime.h>

#include <cmath>
#include <utility>

#include "internal.hpp"
#include "krige_mixed.hpp"

namespace cesim {

// ------------------------------------------------------------ FP64 kernel
// D[r][g] = sum_i X[r][i] K12[g][i] on v_mfma_f64_16x16x4f64 (lane l holds
// A[l % 16][l / 16] and B[l / 16][l % 16]; accumulator v of lane l is
// D[l / 16 + 4 v][l % 16]): grid nodes run along the lanes, so stores are
// runs of 16 consecutive nodes.  Workgroup: 4 waves, 128 nodes x 128
// realizations; wave w owns nodes [32w, 32w + 32) (2 blocks of 16) and all
// 8 blocks of 16 realizations.  Chunks of 16 observations are double-buffered
// in LDS, the next one fetched into registers during the current product.
__global__ void __launch_bounds__(256, 2)
k_krige_f64(double* __restrict__ fields, int m1, int M, int R, const double* __restrict__ X,
            int n, const double2* __restrict__ st, double ux, double uxy, double uyx, double uy,
            double dx, double dy, int nu_code, double sigma2, const int* __restrict__ fail) {
  if (fail[0] & 2) return;   // failed factorisation: the fields stay as drawn
  constexpr int TG = 128, TR = 128, TK = 16;
  __shared__ double Xs[2][TK][TR + 1];
  __shared__ double2 Ss[2][TK];
  const int g0 = blockIdx.x * TG, r0 = blockIdx.y * TR;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double gxt[2], gyt[2];
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const int g = min(g0 + 32 * wave + 16 * t + (lane & 15), M - 1);
    const double gx = (double)(g % m1) * dx, gy = (double)(g / m1) * dy;
    gxt[t] = ux * gx + uxy * gy;
    gyt[t] = uyx * gx + uy * gy;
  }
  doublex4 acc[2][8];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 8; ++b) acc[a][b] = (doublex4){0.0, 0.0, 0.0, 0.0};
  // fetch: thread t loads 8 coefficients of realization row t/2, half t%2
  const int frow = threadIdx.x >> 1, fhalf = (threadIdx.x & 1) * 8;
  double pv[8];
  double2 ps = {0.0, 0.0};
#define CESIM_FETCH64(I0)                                                    \
  {                                                                          \
    const int gr_ = r0 + frow;                                               \
    _Pragma("unroll") for (int u = 0; u < 8; ++u) {                          \
      const int gi_ = (I0) + fhalf + u;                                      \
      pv[u] = (gr_ < R && gi_ < n) ? X[(size_t)gr_ * n + gi_] : 0.0;         \
    }                                                                        \
    if (threadIdx.x < TK) ps = st[min((I0) + (int)threadIdx.x, n - 1)];      \
  }
#define CESIM_STASH64(BUF)                                                   \
  {                                                                          \
    _Pragma("unroll") for (int u = 0; u < 8; ++u) Xs[BUF][fhalf + u][frow] = pv[u]; \
    if (threadIdx.x < TK) Ss[BUF][threadIdx.x] = ps;                         \
  }
  CESIM_FETCH64(0)
  CESIM_STASH64(0)
  __syncthreads();
  const int nchunks = (n + TK - 1) / TK;
  for (int kc = 0; kc < nchunks; ++kc) {
    const int buf = kc & 1;
    if (kc + 1 < nchunks) CESIM_FETCH64((kc + 1) * TK)
#pragma unroll
    for (int ks = 0; ks < TK; ks += 4) {
      const int kk = ks + (lane >> 4);
      const double2 sv = Ss[buf][kk];
      double kg[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const double hx = gxt[t] - sv.x, hy = gyt[t] - sv.y;
        kg[t] = sigma2 * matern_rho(nu_code, sqrt(hx * hx + hy * hy));
      }
#pragma unroll
      for (int b = 0; b < 8; ++b) {
        const double a = Xs[buf][kk][16 * b + (lane & 15)];
#pragma unroll
        for (int t = 0; t < 2; ++t)
          acc[t][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, kg[t], acc[t][b], 0, 0, 0);
      }
    }
    if (kc + 1 < nchunks) CESIM_STASH64(buf ^ 1)
    __syncthreads();
  }
#undef CESIM_FETCH64
#undef CESIM_STASH64
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const int g = g0 + 32 * wave + 16 * t + (lane & 15);
    if (g >= M) continue;
#pragma unroll
    for (int b = 0; b < 8; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = r0 + 16 * b + (lane >> 4) + 4 * v;
        if (r < R) fields[(size_t)r * M + g] += acc[t][b][v];
      }
  }
}

// Kriging prediction from the observed values, yhat[g] = sum_i C(g - s_i)
// chat_i with chat = A^{-1} z (the term K12 (K22 + tau^2 I)^{-1} z of eq. (4),
// common to every realization), in FP64, one grid node per thread, stations
// staged through LDS.  The mixed path adds it to every realization and runs
// its half-precision GEMM on the per-realization part only: with data that
// the covariance does not explain well chat is large and K12 chat cancels
// strongly, which half-precision operands and FP32 sums would not resolve.
// Near pairs -- lag below kNear range units, where the correlation exceeds
// 1e-4 (exp(-x) for nu = 1/2, x sqrt 2 K1(x sqrt 2) for nu = 1,
// (1 + x sqrt 3) exp(-x sqrt 3) for nu = 3/2, each with margin) -- are
// evaluated entirely in FP64.  Far pairs use FP32 coordinates pre-scaled by
// kappa (as in the mixed GEMM) and the FP32 correlation: its relative error
// (a few 1e-6, from the rounded lag) times a correlation below 1e-4 stays far
// below the FP64 terms' rounding in the cancelling sum; they are summed per
// chunk of 256 stations in FP32 and the chunk sums in FP64.  Pairs farther
// than kSkip range units (correlation below 1e-13) are left out: each such
// term is under 1e-13 |chat_i|, a thousandth of the error (a few
// 1e-10 |chat_i|) of one FP32 far term at the near bound.
//
// Work item (x, y, z) is a tile of 32 x 32 grid nodes and the z-th slice
// of `slice` stations in the GEMM's Morton order (position p holds station
// order[p]), staged through LDS kPredStage at a time; its FP64 partial sums
// go to part[z][g], and k_predict_sum adds the slices in order.  Each
// workgroup takes the next item from the counter *next (zero at launch)
// until none is left: items cost more near station clusters, and a fixed
// share per workgroup left the slowest one running alone at the end; the
// sums do not depend on which workgroup computes an item.  Stations come
// in chunks of kGemmChunk with bounding circles: a chunk whose circle is
// farther than kNear range units from the tile's for certain takes the
// FP32 branch for every pair, as the per-pair test would, with no test and
// no divergence, and one farther than kSkip is passed over.  The solves run
// beside the prediction as chains of small kernels; with one workgroup
// (50 KB of LDS, 16 waves) per CU their workgroups find free wave slots at
// once instead of queueing behind prediction tiles.
constexpr int kPredThreads = 1024;
constexpr int kPredStage = 1280;
template <int NU>
__global__ void __launch_bounds__(kPredThreads)
k_predict_f64(double* __restrict__ part, int m1, int m2, int n, int slice, int gx_tiles,
              int gy_tiles, int nitems, const double* __restrict__ chat,
              const double2* __restrict__ st, const int* __restrict__ order,
              const float4* __restrict__ circ, double ux, double uxy, double uyx, double uy,
              double dx, double dy, int* __restrict__ next) {
  constexpr double kNear = NU == 0 ? 9.5 : (NU == 1 ? 8.0 : 7.0);
  constexpr double kKappa = NU == 0 ? kLog2e : (NU == 1 ? kSqrt2 : kSqrt3);
  constexpr float kNearS2 = (float)(kNear * kKappa * kNear * kKappa);
  // far for certain: the lower bound of the scaled lag clears kNear kappa
  // with room for the rounding of the FP32 coordinates and circles
  constexpr float kFarBound = (float)(kNear * kKappa) * 1.0001f + 1e-2f;
  // negligible for certain: beyond kSkip range units every correlation is
  // below 1e-13 (exp(-x) at x = 29.9, x sqrt 2 K1(x sqrt 2) at 22.6,
  // (1 + x sqrt 3) exp(-x sqrt 3) at 19.3)
  constexpr double kSkip = NU == 0 ? 30.5 : (NU == 1 ? 23.0 : 19.8);
  constexpr float kSkipBound = (float)(kSkip * kKappa);
  __shared__ double2 S[kPredStage];
  __shared__ float4 P[kPredStage];   // kappa-scaled FP32 coordinates, chat in FP32
  __shared__ double Cv[kPredStage];
  __shared__ int s_item;
  // work item w: tile (w % gx_tiles, (w / gx_tiles) % gy_tiles), slice
  // w / (gx_tiles gy_tiles); every wave runs the same items
  for (;;) {
  if (threadIdx.x == 0) s_item = atomicAdd(next, 1);
  __syncthreads();
  const int w = s_item;
  __syncthreads();
  if (w >= nitems) break;
  const int tx = w % gx_tiles, ty = (w / gx_tiles) % gy_tiles, tz = w / (gx_tiles * gy_tiles);
  const int ix = tx * 32 + (threadIdx.x & 31), iy = ty * 32 + (threadIdx.x >> 5);
  const double gx = (double)min(ix, m1 - 1) * dx, gy = (double)min(iy, m2 - 1) * dy;
  const double a = ux * gx + uxy * gy, b = uyx * gx + uy * gy;
  const float a32 = (float)(kKappa * a), b32 = (float)(kKappa * b);
  // bounding circle of the tile's nodes in scaled coordinates
  float tcx, tcy, trad;
  {
    const int ia = tx * 32, ib = min(ia + 31, m1 - 1);
    const int ja = ty * 32, jb = min(ja + 31, m2 - 1);
    const double x = 0.5 * (ia + ib) * dx, y = 0.5 * (ja + jb) * dy;
    const double hx = 0.5 * (ib - ia) * dx, hy = 0.5 * (jb - ja) * dy;
    tcx = (float)(kKappa * (ux * x + uxy * y));
    tcy = (float)(kKappa * (uyx * x + uy * y));
    const double px = ux * hx + uxy * hy, py = uyx * hx + uy * hy;   // half-diagonals
    const double qx = ux * hx - uxy * hy, qy = uyx * hx - uy * hy;
    trad = (float)(kKappa * sqrt(fmax(px * px + py * py, qx * qx + qy * qy)));
  }
  double acc = 0.0;
  const int pb = tz * slice, pe = min(n, pb + slice);
  for (int p0 = pb; p0 < pe; p0 += kPredStage) {
    const int cnt = min(kPredStage, pe - p0);
    __syncthreads();
    for (int t = threadIdx.x; t < cnt; t += kPredThreads) {
      const int idx = order[p0 + t];
      const double2 sv = st[idx];
      const double cv = chat[idx];
      S[t] = sv;
      Cv[t] = cv;
      P[t] = make_float4((float)(kKappa * sv.x), (float)(kKappa * sv.y), (float)cv, 0.f);
    }
    __syncthreads();
    for (int b0 = 0; b0 < cnt; b0 += 256) {     // FP32 sums of far pairs per 256 stations
      float far = 0.0f;
      const int be = min(cnt, b0 + 256);
      for (int j0 = b0; j0 < be; j0 += kGemmChunk) {
        const float4 q = circ[(p0 + j0) / kGemmChunk];
        const float ddx = tcx - q.x, ddy = tcy - q.y;
        const float lb = __builtin_amdgcn_sqrtf(ddx * ddx + ddy * ddy) - trad - q.z;
        if (lb > kSkipBound) continue;
        const int je = min(be, j0 + kGemmChunk);
        if (lb > kFarBound) {
#pragma unroll 4
          for (int j = j0; j < je; ++j) {
            const float4 pj = P[j];
            const float hx = a32 - pj.x, hy = b32 - pj.y;
            far = fmaf(rho_scaled_f32(NU, __builtin_amdgcn_sqrtf(hx * hx + hy * hy)), pj.z, far);
          }
        } else {
#pragma unroll 4
          for (int j = j0; j < je; ++j) {
            const float4 pj = P[j];
            const float hx = a32 - pj.x, hy = b32 - pj.y;
            const float xs2 = hx * hx + hy * hy;
            if (xs2 < kNearS2) {
              const double ex = a - S[j].x, ey = b - S[j].y;
              acc = fma(matern_rho(NU, sqrt(ex * ex + ey * ey)), Cv[j], acc);
            } else {
              far = fmaf(rho_scaled_f32(NU, __builtin_amdgcn_sqrtf(xs2)), pj.z, far);
            }
          }
        }
      }
      acc += (double)far;
    }
  }
  if (ix < m1 && iy < m2) part[(size_t)tz * m1 * m2 + (size_t)iy * m1 + ix] = acc;
  }
}

__global__ void k_zero_int(int* __restrict__ v) { *v = 0; }

// yhat[g] = sigma^2 (sum of the S slice sums of node g, in slice order), FP32.
__global__ void __launch_bounds__(256)
k_predict_sum(float* __restrict__ yhat, const double* __restrict__ part, int M, int S,
              double sigma2) {
  const int g = blockIdx.x * 256 + threadIdx.x;
  if (g >= M) return;
  double acc = 0.0;
  for (int q = 0; q < S; ++q) acc += part[(size_t)q * M + g];
  yhat[g] = (float)(sigma2 * acc);
}

// ----------------------------------------------------------- mixed kernel

// Coefficient split, one workgroup per realization r (r < Rp; rows r >= R
// are zero): scale_r = max_i |X[r][i]|, v = X[r][i] / scale_r in [-1, 1],
// hi = half(v), lo = half(v - hi), stored as Bh/Bl[kc][r][32] (observation
// chunk kc of 32, observations in the GEMM's order: position i holds
// observation order[i]).  colscale[r] = scale_r sigma^2 / KS undoes the
// scaling in the GEMM epilogue (KS is the factor the correlations are
// multiplied by before conversion, keeping FP16 values in the normal range).
template <typename H>
__global__ void __launch_bounds__(256)
k_split_coef(const double* __restrict__ X, int n, int R, int Rp, double sigma2, double ks,
             const int* __restrict__ order, H* __restrict__ Bh, H* __restrict__ Bl,
             float* __restrict__ colscale) {
  __shared__ double red[256];
  const int r = blockIdx.x;
  const int npad = (n + kKC - 1) / kKC * kKC;
  double mx = 0.0;
  if (r < R)
    for (int i = threadIdx.x; i < n; i += 256) mx = fmax(mx, fabs(X[(size_t)r * n + i]));
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + h]);
    __syncthreads();
  }
  const double sc = red[0];
  const double inv = sc > 0.0 ? 1.0 / sc : 0.0;
  for (int i = threadIdx.x; i < npad; i += 256) {
    const double v = (i < n && r < R) ? X[(size_t)r * n + order[i]] * inv : 0.0;
    const H h = (H)(float)v;
    const H l = (H)(float)(v - (double)(float)h);
    const size_t o = ((size_t)(i / kKC) * Rp + r) * kKC + (i % kKC);
    Bh[o] = h;
    Bl[o] = l;
  }
  if (threadIdx.x == 0) colscale[r] = (float)(sc * sigma2 / ks);
}

// Same product with a workgroup of 8 waves over 128 grid nodes x 512
// realizations: waves w and w + 4 own the same 32 nodes and realizations
// [r0 + 256 (w / 4), + 256).  The correlations of a chunk of 32 observations
// are computed once per workgroup: wave w / 4 = q evaluates k-step q (16
// observations) for its nodes, keeps it in registers and posts it to LDS,
// and reads the other k-step from its partner -- half the arithmetic per
// matrix instruction of the 4-wave kernel.  The correlations of chunk kc + 1
// are evaluated while chunk kc is multiplied.
template <int NU, typename H>
__global__ void __launch_bounds__(512, 1)
k_krige_split3_x(float* __restrict__ fields, int m1, int M, int R, int Rp,
                 const H* __restrict__ Bh, const H* __restrict__ Bl,
                 const float* __restrict__ colscale, const float* __restrict__ yhat, int n,
                 const float2* __restrict__ st, const float4* __restrict__ circ, float xcut,
                 float ux, float uxy, float uyx, float uy, float dx, float dy, float kscale,
                 const int* __restrict__ fail) {
  if (fail[0] & 2) return;   // failed factorisation: the fields stay as drawn
  using HV = typename HalfOps<H>::V;
  constexpr int TG = 128, TR = 512;
  __shared__ __align__(16) H Sh[2][TR * kKC];
  __shared__ __align__(16) H Sl[2][TR * kKC];
  __shared__ __align__(16) HV Kx[4][2][2][64];     // [node frag][k-step][hi, lo][lane]
  __shared__ float2 Ss[3][kKC];
  const int g0 = blockIdx.x * TG, r0 = blockIdx.y * TR;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nf = wave & 3, q = wave >> 2;
  const bool upper = lane >= 32;
  float gxt[1], gyt[1];
  node_coords(min(g0 + 32 * nf + (lane & 31), M - 1), m1, dx, dy, ux, uxy, uyx, uy, gxt[0],
              gyt[0]);
  floatx16 acc[1][8];
#pragma unroll
  for (int b = 0; b < 8; ++b)
#pragma unroll
    for (int e = 0; e < 16; ++e) acc[0][b][e] = 0.0f;
  const int nchunks = (n + kKC - 1) / kKC;
  u32x4v ph[4], pl[4];
#define CESIM_FETCHX(KC)                                                                    \
  {                                                                                         \
    const u32x4v* gh_ = reinterpret_cast<const u32x4v*>(Bh + ((size_t)(KC) * Rp + r0) * kKC); \
    const u32x4v* gl_ = reinterpret_cast<const u32x4v*>(Bl + ((size_t)(KC) * Rp + r0) * kKC); \
    ph[0] = gh_[threadIdx.x];                                                               \
    ph[1] = gh_[threadIdx.x + 512];                                                         \
    ph[2] = gh_[threadIdx.x + 1024];                                                        \
    ph[3] = gh_[threadIdx.x + 1536];                                                        \
    pl[0] = gl_[threadIdx.x];                                                               \
    pl[1] = gl_[threadIdx.x + 512];                                                         \
    pl[2] = gl_[threadIdx.x + 1024];                                                        \
    pl[3] = gl_[threadIdx.x + 1536];                                                        \
  }
#define CESIM_ST1X(U)                                                     \
  {                                                                       \
    const int qq = threadIdx.x + 512 * (U), row = qq >> 2;                \
    const int pq = (row << 2) | ((qq & 3) ^ ((row >> 2) & 3));            \
    sh_[pq] = ph[U];                                                      \
    sl_[pq] = pl[U];                                                      \
  }
#define CESIM_STASHX(BUF)                                                 \
  {                                                                       \
    u32x4v* sh_ = reinterpret_cast<u32x4v*>(Sh[BUF]);                     \
    u32x4v* sl_ = reinterpret_cast<u32x4v*>(Sl[BUF]);                     \
    CESIM_ST1X(0) CESIM_ST1X(1) CESIM_ST1X(2) CESIM_ST1X(3)               \
  }
  // the chunks whose split correlations with the tile are all exact zeros
  // are skipped, as in the 4-wave kernel (uniform over the workgroup)
  float tcx, tcy, trad;
  tile_circle(g0, TG, M, m1, dx, dy, ux, uxy, uyx, uy, tcx, tcy, trad);
  auto next_live = [&](int kc) {
    for (; kc < nchunks; ++kc) {
      const float4 c4 = circ[kc];
      const float ddx = tcx - c4.x, ddy = tcy - c4.y;
      if (__builtin_amdgcn_sqrtf(ddx * ddx + ddy * ddy) - trad - c4.z < xcut) break;
    }
    return kc;
  };
  // stations rotate through three chunk buffers as in the 4-wave kernel:
  // the current live chunk, the next (its correlations are formed during
  // the current one's products) and the one after (its stations loaded)
  const int sl_ = threadIdx.x & (kKC - 1);
  int cur = next_live(0), nxt = next_live(cur + 1);
  Ss[0][sl_] = st[min(cur * kKC + sl_, n - 1)];
  Ss[1][sl_] = st[min(nxt * kKC + sl_, n - 1)];
  CESIM_FETCHX(min(cur, nchunks - 1))
  CESIM_STASHX(0)
  __syncthreads();
  HV own_h[1], own_l[1], oth_h[1], oth_l[1];
  k12_step<NU, 1, H>(Ss[0] + 16 * q, upper, gxt, gyt, kscale, own_h, own_l);
  Kx[nf][q][0][lane] = own_h[0];
  Kx[nf][q][1][lane] = own_l[0];
  __syncthreads();
  for (int it = 0; cur < nchunks; ++it) {
    const int buf = it & 1;
    const int sb = it % 3, sb1 = sb == 2 ? 0 : sb + 1, sb2 = sb1 == 2 ? 0 : sb1 + 1;
    const int nn = next_live(nxt + 1);
    oth_h[0] = Kx[nf][1 - q][0][lane];
    oth_l[0] = Kx[nf][1 - q][1][lane];
    CESIM_FETCHX(min(nxt, nchunks - 1))
    const float2 ps = st[min(nn * kKC + sl_, n - 1)];
    // k-step 0 is wave group 0's correlations, k-step 1 group 1's
    if (q == 0) {
      mfma_step<1, H>(Sh[buf] + 256 * q * kKC, Sl[buf] + 256 * q * kKC, 0, lane, own_h, own_l, acc);
      mfma_step<1, H>(Sh[buf] + 256 * q * kKC, Sl[buf] + 256 * q * kKC, 16, lane, oth_h, oth_l, acc);
    } else {
      mfma_step<1, H>(Sh[buf] + 256 * q * kKC, Sl[buf] + 256 * q * kKC, 0, lane, oth_h, oth_l, acc);
      mfma_step<1, H>(Sh[buf] + 256 * q * kKC, Sl[buf] + 256 * q * kKC, 16, lane, own_h, own_l, acc);
    }
    k12_step<NU, 1, H>(Ss[sb1] + 16 * q, upper, gxt, gyt, kscale, own_h, own_l);
    __syncthreads();                                   // Kx and Sh/Sl[buf ^ 1] free
    Kx[nf][q][0][lane] = own_h[0];
    Kx[nf][q][1][lane] = own_l[0];
    CESIM_STASHX(buf ^ 1)
    Ss[sb2][sl_] = ps;
    __syncthreads();
    cur = nxt;
    nxt = nn;
  }
#undef CESIM_FETCHX
#undef CESIM_STASHX
#undef CESIM_ST1X
  const int gg = g0 + 32 * nf + (lane & 31);
  if (gg >= M) return;
  const float yh = yhat[gg];
  const int rq = r0 + 256 * q;
#pragma unroll
  for (int b = 0; b < 8; ++b)
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int r = rq + 32 * b + 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3);
      if (r < R) fields[(size_t)r * M + gg] += fmaf(acc[0][b][e], colscale[r], yh);
    }
}

// The FP32 comparison variant of the mixed grid product (no split):
// coefficients transposed to [observation][Rp] in FP32 (scaled by sigma^2),
// observations in the original order, rows >= n zero.
__global__ void __launch_bounds__(256)
k_coef_f32(const double* __restrict__ X, int n, int R, int Rp, int npad, double sigma2,
           float* __restrict__ Xf) {
  const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (size_t)npad * Rp) return;
  const int i = (int)(e / Rp), r = (int)(e % Rp);
  Xf[e] = (i < n && r < R) ? (float)(X[(size_t)r * n + i] * sigma2) : 0.0f;
}

// Grid product in FP32 on matrix cores, v_mfma_f32_32x32x2f32: lane l holds
// A[l % 32][l / 32] and B[l / 32][l % 32]; the accumulator layout is that of
// the 32x32x16 kernels.  The product is formed transposed, D[r][g] = sum_i
// X[r][i] K12[g][i], so the accumulator lanes run over grid nodes.
// Workgroup: 4 waves, 128 nodes x 256 realizations; wave w owns nodes
// [32 w, 32 w + 32) and all 8 blocks of 32 realizations.  Per pair of
// observations a lane evaluates one FP32 correlation (its node, observation
// l / 32) for 8 matrix instructions.  Coefficient chunks of 32 observations
// are double-buffered in LDS as [observation][realization].
template <int NU>
__global__ void __launch_bounds__(256, 2)
k_krige_fp32(float* __restrict__ fields, int m1, int M, int R, int Rp,
             const float* __restrict__ Xf, const float* __restrict__ yhat, int n,
             const float2* __restrict__ st, float ux, float uxy, float uyx, float uy, float dx,
             float dy, const int* __restrict__ fail) {
  if (fail[0] & 2) return;   // failed factorisation: the fields stay as drawn
  constexpr int TR = 256, KC = 32;
  __shared__ __align__(16) float Xs[2][KC][TR];
  __shared__ float2 Ss[2][KC];
  const int g0 = blockIdx.x * 128, r0 = blockIdx.y * TR;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  float gxt, gyt;
  node_coords(min(g0 + 32 * wave + (lane & 31), M - 1), m1, dx, dy, ux, uxy, uyx, uy, gxt, gyt);
  floatx16 acc[8];
#pragma unroll
  for (int b = 0; b < 8; ++b)
#pragma unroll
    for (int e = 0; e < 16; ++e) acc[b][e] = 0.0f;
  const int nchunks = (n + KC - 1) / KC;
  u32x4v pv[8];
  float2 ps = {0.f, 0.f};
  // 16-byte piece q = t + 256 u of a chunk: observation q / 64, realizations
  // 4 (q % 64) .. + 3
  auto fetch = [&](int kc) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int q = threadIdx.x + 256 * u;
      pv[u] = *reinterpret_cast<const u32x4v*>(Xf + (size_t)(kc * KC + (q >> 6)) * Rp + r0 +
                                               4 * (q & 63));
    }
    if (threadIdx.x < KC) ps = st[min(kc * KC + (int)threadIdx.x, n - 1)];
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int q = threadIdx.x + 256 * u;
      *reinterpret_cast<u32x4v*>(&Xs[buf][q >> 6][4 * (q & 63)]) = pv[u];
    }
    if (threadIdx.x < KC) Ss[buf][threadIdx.x] = ps;
  };
  fetch(0);
  stash(0);
  __syncthreads();
  for (int kc = 0; kc < nchunks; ++kc) {
    const int buf = kc & 1;
    if (kc + 1 < nchunks) fetch(kc + 1);
#pragma unroll
    for (int kk = 0; kk < KC; kk += 2) {
      const int k = kk + (lane >> 5);
      const float2 s = Ss[buf][k];
      const float hx = gxt - s.x, hy = gyt - s.y;
      const float kg = rho_scaled_f32(NU, __builtin_amdgcn_sqrtf(hx * hx + hy * hy));
#pragma unroll
      for (int b = 0; b < 8; ++b)
        acc[b] = __builtin_amdgcn_mfma_f32_32x32x2f32(Xs[buf][k][32 * b + (lane & 31)], kg, acc[b],
                                                      0, 0, 0);
    }
    if (kc + 1 < nchunks) stash(buf ^ 1);
    __syncthreads();
  }
  const int gg = g0 + 32 * wave + (lane & 31);
  if (gg >= M) return;
  const float yh = yhat[gg];
#pragma unroll
  for (int b = 0; b < 8; ++b)
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int r = r0 + 32 * b + 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3);
      if (r < R) fields[(size_t)r * M + gg] += acc[b][e] + yh;
    }
}

// ------------------------------------------------------------------- host


// Linear map U (range units) and the per-path coordinate scale.
static void cov_map(const cesim_ctx c, double scale, double& ux, double& uxy, double& uyx,
                    double& uy) {
  ux = c->covd.u00 * scale;
  uxy = c->covd.u01 * scale;
  uyx = c->covd.u10 * scale;
  uy = c->covd.u11 * scale;
}

// Scaled distance beyond which every correlation, multiplied by ks and
// rounded to FP16 in the split, is zero (with an 8x margin below half the
// smallest FP16 subnormal, 2^-25), from upper bounds of the correlation in
// the kernel's scaled distance x: 2^-x (nu = 1/2), (1 + x) e^-x (nu = 3/2),
// sqrt(pi x / 2) e^-x (1 + 1/(2x)) (nu = 1, from the asymptotic expansion
// of K_1).  ks = 0 (BF16, whose range keeps every such value): no cut-off.
static double split_cutoff(int nu_code, double ks) {
  if (ks <= 0.0) return 1e30;
  const double lim = std::ldexp(1.0, -28) / ks;
  auto bound = [&](double x) {
    if (nu_code == 0) return std::exp2(-x);
    if (nu_code == 2) return (1.0 + x) * std::exp(-x);
    return std::sqrt(M_PI * x / 2.0) * std::exp(-x) * (1.0 + 0.5 / x);
  };
  double x = 8.0;
  while (bound(x) >= lim) x += 0.25;
  return x + 0.5;
}

// Coefficient buffers for R realizations: [R][n] FP64 and, on the mixed
// path, the half-precision hi / lo split with its column scales.
cesim_status krige_reserve(cesim_ctx c, int R) {
  const int n = c->nobs;
  CESIM_TRY(c->coef.reserve(sizeof(double) * (size_t)n * R));
  CESIM_TRY(c->solve_tmp.reserve(sizeof(double) * (size_t)n * R));
  if (c->prec == CESIM_PREC_MIXED) {
    const int Rp = (R + 511) / 512 * 512;        // covers every GEMM tile
    const int npad = (n + kKC - 1) / kKC * kKC;
    CESIM_TRY(c->coef_b16.reserve(sizeof(uint16_t) * 2 * (size_t)npad * Rp + sizeof(float) * Rp));
  }
  return CESIM_OK;
}

static cesim_status predict_from_chat(cesim_ctx c, hipStream_t s);

// aux waits for the last kernel of the previous condition() that read the
// factor, the observed values or the prediction (once per condition()).
cesim_status aux_wait_last_use(cesim_ctx c) {
  if (c->last_use_valid) {
    CESIM_HIP(hipStreamWaitEvent(c->aux, c->last_use, 0));
    c->last_use_valid = false;
  }
  return CESIM_OK;
}

// Everything is queued before the host waits, the work of the stream first
// where it does not depend on aux (launches reach the GPU only as fast as
// a long dependent chain on aux retires them): with joint sampling the box
// factors on aux, then on the stream the synthetic data, then on aux the
// factorisation (when the nugget or the stations changed), the mixed path's
// prediction on the look-ahead stream, the solves on the stream after
// factor_ready, and the grid GEMM after the prediction and aux_done.  A new
// prediction (chat = A^{-1} z by its own one-vector solve, then yhat)
// follows the factorisation and runs beside the solves rather than after
// them.  Only then do the factorisations' status come back to the host;
// after a failed pivot the GEMM has left the fields unchanged.
cesim_status condition_device(cesim_ctx c, double nugget, void* fields) {
  hipStream_t s = c->stream;
  const int R = c->nreal;
  const bool mixed = c->prec == CESIM_PREC_MIXED;
  if (joint_active(c) && c->max_box > kMaxJointBox) return CESIM_ERR_INVALID_ARG;
  const bool refactor = !c->chol_valid || c->chol_nugget != nugget;
  const bool boxes = joint_active(c) && (refactor || !c->box_fac_valid);
  const bool predict = mixed && (refactor || !c->yhat_valid);
  if (refactor) c->chol_valid = false;
  if (predict) c->yhat_valid = false;
  if (refactor || boxes || predict) CESIM_TRY(aux_wait_last_use(c));
  if (refactor || boxes) CESIM_HIP(hipMemsetAsync(c->chol_info.p, 0, sizeof(int) * 4, c->aux));
  if (boxes) {
    c->box_fac_valid = false;
    CESIM_TRY(box_factor_device(c, nugget, c->aux));
    if (!refactor)
      CESIM_HIP(hipMemcpyAsync(c->chol_info_host, c->chol_info.p, sizeof(int) * 4,
                               hipMemcpyDeviceToHost, c->aux));
    CESIM_HIP(hipEventRecord(c->box_ready, c->aux));
  }
  CESIM_TRY(lk_phi_device(c, nugget));
  CESIM_TRY(krige_reserve(c, R));
  double* X = c->coef.as<double>();
  // FP64: X = A^{-1} (z - z*_r); mixed: X = -A^{-1} z*_r (yhat carries z)
  if (!mixed && c->z_pending) CESIM_HIP(hipStreamWaitEvent(s, c->z_ready, 0));
  c->z_pending = false;
  if (boxes) CESIM_HIP(hipStreamWaitEvent(s, c->box_ready, 0));
  CESIM_TRY(lk_synth_rhs_device(c, fields, X, !mixed));
  if (refactor) {
    CESIM_TRY(chol_factor_device(c, nugget, c->aux, false));
    CESIM_HIP(hipEventRecord(c->factor_ready, c->aux));
    CESIM_HIP(hipStreamWaitEvent(s, c->factor_ready, 0));
  }
  if (predict) {
    // the prediction follows the factor on the look-ahead stream (idle by
    // then), and is queued before the solves: each launch costs the host
    // about as long as the GPU takes to run it, so a chain queued after the
    // solves starts only as they end
    CESIM_HIP(hipEventRecord(c->la_panel, c->aux));
    CESIM_HIP(hipStreamWaitEvent(c->look, c->la_panel, 0));
    CESIM_TRY(predict_device(c, c->look));
    CESIM_HIP(hipEventRecord(c->la_update, c->look));
  }
  // A later call of at most kInverseMaxReal realizations on the same factor
  // (mixed path) takes the coefficients from one GEMM with A^{-1}, formed on
  // the first such call: streams of small calls then skip the substitutions'
  // chain of dependent launches, which costs such a call about as much as
  // its grid GEMM.  Larger calls and the first call after a factorisation
  // run the substitutions (forming A^{-1} costs about three chains).
  if (mixed && !refactor && R <= kInverseMaxReal && c->nobs <= kInverseMaxObs) {
    if (!c->ainv_valid) CESIM_TRY(inverse_device(c, s));
    CESIM_TRY(apply_inverse_device(c, X, R, c->solve_tmp.as<double>(), s));
    std::swap(c->coef, c->solve_tmp);
    X = c->coef.as<double>();
  } else {
    CESIM_TRY(chol_solve_device(c, X, R, s, c->solve_tmp.as<double>()));
  }
  if (predict) CESIM_HIP(hipStreamWaitEvent(s, c->la_update, 0));
  if (c->aux_pending) {
    CESIM_HIP(hipEventRecord(c->aux_done, c->aux));
    CESIM_HIP(hipStreamWaitEvent(s, c->aux_done, 0));
    c->aux_pending = false;
  }
  CESIM_TRY(krige_grid_device(c, X, fields));
  CESIM_HIP(hipEventRecord(c->last_use, s));
  c->last_use_valid = true;
  if (refactor || boxes) {
    CESIM_HIP(hipEventSynchronize(refactor ? c->factor_ready : c->box_ready));
    if (c->chol_info_host[0] & 2) {
      c->yhat_valid = false;
      c->chol_valid = false;
      return CESIM_ERR_NOT_POSITIVE_DEFINITE;
    }
    if (boxes) c->box_fac_valid = true;
    c->chol_valid = true;
    c->chol_nugget = nugget;
  }
  return CESIM_OK;
}

// The FP32 comparison variant (CESIM_PARAM_GEMM_SPLIT = 2) of the mixed
// grid product.
static cesim_status krige_grid_fp32(cesim_ctx c, const double* X, float* fields) {
  hipStream_t s = c->stream;
  const int n = c->nobs, R = c->nreal, m1 = c->grid.m1, M = c->grid.m1 * c->grid.m2;
  const int Rp = (R + 255) / 256 * 256, npad = (n + 31) / 32 * 32;
  CESIM_TRY(krige_reserve(c, R));
  float* Xf = c->coef_b16.as<float>();          // 2 x 2 bytes per entry reserved: fits FP32
  int tr = c->timer.begin(ST_COEF_SPLIT, s);
  const size_t tot = (size_t)npad * Rp;
  k_coef_f32<<<(unsigned)((tot + 255) / 256), 256, 0, s>>>(X, n, R, Rp, npad, c->covd.sigma2, Xf);
  CESIM_HIP(hipGetLastError());
  c->timer.end(tr, s);
  const double kappa = c->covd.nu_code == 0 ? kLog2e : (c->covd.nu_code == 2 ? kSqrt3 : kSqrt2);
  double ux, uxy, uyx, uy;
  cov_map(c, kappa, ux, uxy, uyx, uy);
  const dim3 grid((M + 127) / 128, Rp / 256);
  const float a = (float)ux, b = (float)uxy, cc = (float)uyx, d = (float)uy;
  const float fdx = (float)c->grid.dx, fdy = (float)c->grid.dy;
  const float2* S2 = c->obs_t32.as<float2>();   // original order, as Xf
  const float* YH = c->yhat.as<float>();
  const int* FAIL = c->chol_info.as<int>();
  tr = c->timer.begin(ST_KRIGE_GEMM, s);
  switch (c->covd.nu_code) {
    case 0: k_krige_fp32<0><<<grid, 256, 0, s>>>(fields, m1, M, R, Rp, Xf, YH, n, S2, a, b, cc, d, fdx, fdy, FAIL); break;
    case 1: k_krige_fp32<1><<<grid, 256, 0, s>>>(fields, m1, M, R, Rp, Xf, YH, n, S2, a, b, cc, d, fdx, fdy, FAIL); break;
    default: k_krige_fp32<2><<<grid, 256, 0, s>>>(fields, m1, M, R, Rp, Xf, YH, n, S2, a, b, cc, d, fdx, fdy, FAIL); break;
  }
  CESIM_HIP(hipGetLastError());
  c->timer.end(tr, s);
  return CESIM_OK;
}

// fields[r] += K12 X[r] for the c->nreal realizations of the last draw
// (Section 2, step 5), FP64 or three-product half-precision split.
cesim_status krige_grid_device(cesim_ctx c, const double* X, void* fields) {
  hipStream_t s = c->stream;
  const int n = c->nobs, R = c->nreal;
  const int m1 = c->grid.m1, M = c->grid.m1 * c->grid.m2;
  const double dx = c->grid.dx, dy = c->grid.dy;
  if (c->prec == CESIM_PREC_FP64) {
    double ux, uxy, uyx, uy;
    cov_map(c, 1.0, ux, uxy, uyx, uy);
    dim3 grid((M + 127) / 128, (R + 127) / 128);
    const int tr = c->timer.begin(ST_KRIGE_GEMM, s);
    k_krige_f64<<<grid, 256, 0, s>>>(static_cast<double*>(fields), m1, M, R, X, n,
                                     c->obs_t64.as<double2>(), ux, uxy, uyx, uy, dx, dy,
                                     c->covd.nu_code, c->covd.sigma2, c->chol_info.as<int>());
    CESIM_HIP(hipGetLastError());
    c->timer.end(tr, s);
    return CESIM_OK;
  }
  if (c->gemm_split == 2) return krige_grid_fp32(c, X, static_cast<float*>(fields));
  const int tile = gemm_tile(c, R);
  // realizations per workgroup tile (tiles 4 and 5: calls of few realizations)
  const int TRr = tile == 3 ? 512 : (tile == 4 ? 64 : (tile == 5 ? 128 : 256));
  const int Rp = (R + TRr - 1) / TRr * TRr;
  const int npad = (n + kKC - 1) / kKC * kKC;
  const bool f16 = c->gemm_split == 0;
  // correlations enter FP16 multiplied by 2^12 (values up to 4096), which
  // keeps products of small correlations out of the subnormal range
  const double ks = f16 ? 4096.0 : 1.0;
  CESIM_TRY(krige_reserve(c, R));
  uint16_t* Hh = c->coef_b16.as<uint16_t>();
  uint16_t* Hl = Hh + (size_t)npad * Rp;
  float* colscale = reinterpret_cast<float*>(Hl + (size_t)npad * Rp);
  int tr = c->timer.begin(ST_COEF_SPLIT, s);
  const int* order = c->obs_order.as<int>();
  if (f16)
    k_split_coef<_Float16><<<Rp, 256, 0, s>>>(X, n, R, Rp, c->covd.sigma2, ks, order,
                                              reinterpret_cast<_Float16*>(Hh),
                                              reinterpret_cast<_Float16*>(Hl), colscale);
  else
    k_split_coef<__bf16><<<Rp, 256, 0, s>>>(X, n, R, Rp, c->covd.sigma2, ks, order,
                                            reinterpret_cast<__bf16*>(Hh),
                                            reinterpret_cast<__bf16*>(Hl), colscale);
  CESIM_HIP(hipGetLastError());
  c->timer.end(tr, s);
  const double kappa = c->covd.nu_code == 0 ? kLog2e : (c->covd.nu_code == 2 ? kSqrt3 : kSqrt2);
  double ux, uxy, uyx, uy;
  cov_map(c, kappa, ux, uxy, uyx, uy);
  tr = c->timer.begin(ST_KRIGE_GEMM, s);
  float* F = static_cast<float*>(fields);
  const float2* S2 = c->obs_t32s.as<float2>();        // the GEMM's station order
  const float4* CIRC = c->gemm_circ.as<float4>();
  const float xcut = (float)split_cutoff(c->covd.nu_code, f16 ? ks : 0.0);
  const float* YH = c->yhat.as<float>();
  const float a = (float)ux, b = (float)uxy, cc = (float)uyx, d = (float)uy;
  const float fdx = (float)dx, fdy = (float)dy, fks = (float)ks;
  const int* FAIL = c->chol_info.as<int>();
  const int nf = tile == 2 ? 2 : 1;
  dim3 grid((M + 128 * nf - 1) / (128 * nf), Rp / TRr);
  const dim3 gridx((M + 127) / 128, Rp / 512);
#define CESIM_KS(NU, NF, NB, H)                                                                 \
  k_krige_split3<NU, NF, NB, H><<<grid, 256, 0, s>>>(                                           \
      F, m1, M, R, Rp, reinterpret_cast<const H*>(Hh), reinterpret_cast<const H*>(Hl), colscale, \
      YH, n, S2, CIRC, xcut, a, b, cc, d, fdx, fdy, fks, FAIL)
#define CESIM_KS_NU(NF, NB, H)                  \
  switch (c->covd.nu_code) {                    \
    case 0: CESIM_KS(0, NF, NB, H); break;      \
    case 1: CESIM_KS(1, NF, NB, H); break;      \
    default: CESIM_KS(2, NF, NB, H); break;     \
  }
#define CESIM_KX(NU, H)                                                                         \
  k_krige_split3_x<NU, H><<<gridx, 512, 0, s>>>(F, m1, M, R, Rp, reinterpret_cast<const H*>(Hh),  \
                                                reinterpret_cast<const H*>(Hl), colscale, YH, n,  \
                                                S2, CIRC, xcut, a, b, cc, d, fdx, fdy, fks, FAIL)
#define CESIM_KX_NU(H)                      \
  switch (c->covd.nu_code) {                \
    case 0: CESIM_KX(0, H); break;          \
    case 1: CESIM_KX(1, H); break;          \
    default: CESIM_KX(2, H); break;         \
  }
  if (tile == 3) {
    if (f16) { CESIM_KX_NU(_Float16) } else { CESIM_KX_NU(__bf16) }
  } else if (nf == 2) {
    if (f16) { CESIM_KS_NU(2, 8, _Float16) } else { CESIM_KS_NU(2, 8, __bf16) }
  } else {
    CESIM_TRY(launch_split3_one_fragment(c->covd.nu_code, tile == 4 ? 2 : (tile == 5 ? 4 : 8), f16,
                                         grid, s, F, m1, M, R, Rp, Hh, Hl, colscale, YH, n, S2,
                                         CIRC, xcut, a, b, cc, d, fdx, fdy, fks, FAIL));
  }
#undef CESIM_KX_NU
#undef CESIM_KX
#undef CESIM_KS_NU
#undef CESIM_KS
  CESIM_HIP(hipGetLastError());
  c->timer.end(tr, s);
  return CESIM_OK;
}

// Mixed path: chat = A^{-1} z and yhat = K12 chat (FP64, stored FP32), once
// per factorisation and set of observed values.
__global__ void k_coef_out(const double* __restrict__ X, const double* __restrict__ chat, int n,
                           size_t total, double* __restrict__ out) {
  const size_t q = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (q < total) out[q] = X[q] + (chat ? chat[q % n] : 0.0);
}

// B_r = A^{-1} (z - z*_r) of the last condition() into out ([R][n]): X
// itself on the FP64 path, chat + X on the mixed path.
cesim_status copy_coefficients_device(cesim_ctx c, double* out) {
  const size_t total = (size_t)c->nobs * c->nreal;
  const double* ch = c->prec == CESIM_PREC_MIXED ? c->chat.as<double>() : nullptr;
  k_coef_out<<<(unsigned)((total + 255) / 256), 256, 0, c->stream>>>(c->coef.as<double>(), ch,
                                                                     c->nobs, total, out);
  CESIM_HIP(hipGetLastError());
  return CESIM_OK;
}

// yhat from c->chat (already A^{-1} z), on stream s.
static cesim_status predict_from_chat(cesim_ctx c, hipStream_t s) {
  const int n = c->nobs, m1 = c->grid.m1, M = c->grid.m1 * c->grid.m2;
  // slices of up to one LDS stage (a multiple of 256 stations), at most 16
  const int nslice = std::min(16, (n + kPredStage - 1) / kPredStage);
  const int slice = ((n + nslice - 1) / nslice + 255) / 256 * 256;
  const int S = (n + slice - 1) / slice;
  CESIM_TRY(c->yhat.reserve(sizeof(float) * M));
  CESIM_TRY(c->pred_part.reserve(sizeof(double) * (size_t)S * M));
  double ux, uxy, uyx, uy;
  cov_map(c, 1.0, ux, uxy, uyx, uy);
  const int tr = c->timer.begin(ST_PREDICT, s);
  const int m2 = c->grid.m2;
  // one workgroup per CU, each looping over tiles x slices: half of each
  // CU's wave slots and most of its LDS stay free for the solves' GEMMs
  // and the draw, which then start without waiting for prediction tiles
  const int gxt = (m1 + 31) / 32, gyt = (m2 + 31) / 32;
  const int nitems = gxt * gyt * S;
  const int nwg = std::min(nitems, std::max(1, c->num_cu));
  double* part = c->pred_part.as<double>();
  CESIM_TRY(c->pred_next.reserve(sizeof(int)));
  int* next = c->pred_next.as<int>();
  k_zero_int<<<1, 1, 0, s>>>(next);
#define CESIM_PRED(NU)                                                                        \
  k_predict_f64<NU><<<nwg, kPredThreads, 0, s>>>(                                             \
      part, m1, m2, n, slice, gxt, gyt, nitems, c->chat.as<double>(), c->obs_t64.as<double2>(), \
      c->obs_order.as<int>(), c->gemm_circ.as<float4>(), ux, uxy, uyx, uy, c->grid.dx, c->grid.dy, \
      next)
  switch (c->covd.nu_code) {
    case 0: CESIM_PRED(0); break;
    case 1: CESIM_PRED(1); break;
    default: CESIM_PRED(2); break;
  }
#undef CESIM_PRED
  CESIM_HIP(hipGetLastError());
  k_predict_sum<<<(M + 255) / 256, 256, 0, s>>>(c->yhat.as<float>(), part, M, S,
                                                c->covd.sigma2);
  CESIM_HIP(hipGetLastError());
  c->timer.end(tr, s);
  c->yhat_valid = true;
  return CESIM_OK;
}

// Mixed path: chat = A^{-1} z and yhat = K12 chat (FP64, stored FP32) on
// stream s, once per factorisation and set of observed values.
cesim_status predict_device(cesim_ctx c, hipStream_t s) {
  if (c->yhat_valid) return CESIM_OK;
  const int n = c->nobs;
  CESIM_TRY(c->chat.reserve(sizeof(double) * n));
  CESIM_TRY(c->chat_tmp.reserve(sizeof(double) * n));
  CESIM_TRY(chol_solve_vec_device(c, c->zdev.as<double>(), c->chat.as<double>(), s,
                                  c->chat_tmp.as<double>(), ST_PREDICT));
  return predict_from_chat(c, s);
}

}  // namespace cesim
