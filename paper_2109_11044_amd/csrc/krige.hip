// krige.hip -- Kriging of the residual coefficients onto the grid (step 5 of
// Section 2; the grid prediction of eq. (4), Section 3):
//   v_r[g] = y_r[g] + sum_i C(g - s_i) B[r][i],
// a dense contraction over the observations whose left factor K12 is far too
// large to store (M x n), so every workgroup generates its K12 tile in
// registers, directly in the matrix-core operand layout, from transformed
// coordinates: x = |U g - U s| is the lag length in range units.
//
//   FP64 path : v_mfma_f64_16x16x4f64, K12 and B in FP64.
//   mixed path: K12 in FP32, split into bf16 hi + lo; B split likewise (with
//               sigma^2 folded in); three v_mfma_f32_32x32x16_bf16 products
//               hi.hi + hi.lo + lo.hi accumulate in FP32.
#include <hip/hip_runtime.h>

#include "internal.hpp"

namespace cesim {

typedef double doublex4 __attribute__((ext_vector_type(4)));
typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// ------------------------------------------------------------ FP64 kernel
// Workgroup: 4 waves, tile 128 grid nodes x 64 realizations; wave w owns
// nodes [32w, 32w + 32) as 2 x 4 blocks of 16 x 16.  k-chunks of 16
// observations are staged in LDS (coefficients and coordinates).
__global__ void __launch_bounds__(256)
k_krige_f64(double* __restrict__ fields, int m1, int M, int R, const double* __restrict__ X,
            int n, const double2* __restrict__ st, double ux, double uxy, double uyx, double uy,
            double dx, double dy, int nu_code, double sigma2) {
  constexpr int TG = 128, TR = 64, TK = 16;
  __shared__ double Bs[TK][TR + 2];
  __shared__ double2 Ss[TK];
  const int g0 = blockIdx.x * TG, r0 = blockIdx.y * TR;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // transformed coordinates of this lane's two grid nodes
  double gxt[2], gyt[2];
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const int g = min(g0 + 32 * wave + 16 * t + (lane & 15), M - 1);
    const double gx = (double)(g % m1) * dx, gy = (double)(g / m1) * dy;
    gxt[t] = ux * gx + uxy * gy;
    gyt[t] = uyx * gx + uy * gy;
  }
  doublex4 acc[2][4];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = (doublex4){0.0, 0.0, 0.0, 0.0};
  for (int i0 = 0; i0 < n; i0 += TK) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = threadIdx.x + 256 * u;
      const int kk = e % TK, rr = e / TK;
      const int gi = i0 + kk, gr = r0 + rr;
      Bs[kk][rr] = (gi < n && gr < R) ? X[(size_t)gr * n + gi] : 0.0;
    }
    if (threadIdx.x < TK) {
      const int gi = i0 + threadIdx.x;
      Ss[threadIdx.x] = gi < n ? st[gi] : st[n - 1];
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < TK; ks += 4) {
      const int kk = ks + (lane >> 4);
      const double2 sv = Ss[kk];
      double a[2], b[4];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const double hx = gxt[t] - sv.x, hy = gyt[t] - sv.y;
        a[t] = sigma2 * matern_rho(nu_code, sqrt(hx * hx + hy * hy));
      }
#pragma unroll
      for (int t = 0; t < 4; ++t) b[t] = Bs[kk][16 * t + (lane & 15)];
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y)
          acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[x], b[y], acc[x][y], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int g = g0 + 32 * wave + 16 * x + (lane >> 4) + 4 * v;   // D[l/16 + 4v][l%16]
        const int r = r0 + 16 * y + (lane & 15);
        if (g < M && r < R) fields[(size_t)r * M + g] += acc[x][y][v];
      }
}

// ----------------------------------------------------------- mixed kernel
// B split: Bh/Bl[kc][r][16] bf16 (observation chunk kc of 16, realization r)
// from FP64 X[r][i] with sigma^2 folded in.
__global__ void k_split_coef(const double* __restrict__ X, int n, int R, int Rp, double scale,
                             __bf16* __restrict__ Bh, __bf16* __restrict__ Bl) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  const int npad = (n + 15) / 16 * 16;
  if (i >= npad) return;
  const double v = (i < n && r < R) ? scale * X[(size_t)r * n + i] : 0.0;
  const float f = (float)v;
  const __bf16 h = (__bf16)f;
  const __bf16 l = (__bf16)(float)(v - (double)(float)h);
  const size_t o = ((size_t)(i / 16) * Rp + r) * 16 + (i % 16);
  Bh[o] = h;
  Bl[o] = l;
}

// Workgroup: 4 waves, tile 128 grid nodes x 256 realizations; wave w owns
// nodes [32w, 32w + 32) x all 256 realizations as 8 blocks of 32 x 32.
// Per chunk of 16 observations each lane evaluates 8 correlations.
// Coordinates are pre-scaled so that rho_scaled_f32 applies directly.
__global__ void __launch_bounds__(256)
k_krige_bf16x3(float* __restrict__ fields, int m1, int M, int R, int Rp,
               const __bf16* __restrict__ Bh, const __bf16* __restrict__ Bl, int n,
               const float2* __restrict__ st, float ux, float uxy, float uyx, float uy, float dx,
               float dy, int nu_code) {
  constexpr int TG = 128, TR = 256, TK = 16;
  __shared__ __align__(16) __bf16 Sh[TR * TK];
  __shared__ __align__(16) __bf16 Sl[TR * TK];
  __shared__ float2 Ss[TK];
  const int g0 = blockIdx.x * TG, r0 = blockIdx.y * TR;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = min(g0 + 32 * wave + (lane & 31), M - 1);
  const float gx = (float)(g % m1) * dx, gy = (float)(g / m1) * dy;
  const float gxt = ux * gx + uxy * gy, gyt = uyx * gx + uy * gy;
  const int kb = (lane >> 5) * 8;
  floatx16 acc[8];
#pragma unroll
  for (int b = 0; b < 8; ++b)
#pragma unroll
    for (int e = 0; e < 16; ++e) acc[b][e] = 0.0f;
  const int nchunks = (n + TK - 1) / TK;
  const int rvalid = min(TR, Rp - r0);
  for (int kc = 0; kc < nchunks; ++kc) {
    // stage B chunk: rows r0 .. r0+TR of 16 bf16 each (contiguous per chunk)
    const uint4* gh = reinterpret_cast<const uint4*>(Bh + ((size_t)kc * Rp + r0) * TK);
    const uint4* gl = reinterpret_cast<const uint4*>(Bl + ((size_t)kc * Rp + r0) * TK);
    uint4* sh = reinterpret_cast<uint4*>(Sh);
    uint4* sl = reinterpret_cast<uint4*>(Sl);
    for (int e = threadIdx.x; e < TR * 2; e += 256) {
      const bool ok = (e >> 1) < rvalid;
      sh[e] = ok ? gh[e] : make_uint4(0, 0, 0, 0);
      sl[e] = ok ? gl[e] : make_uint4(0, 0, 0, 0);
    }
    if (threadIdx.x < TK) {
      const int gi = kc * TK + threadIdx.x;
      Ss[threadIdx.x] = st[min(gi, n - 1)];
    }
    __syncthreads();
    bf16x8 ah, al;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const float2 sv = Ss[kb + j];
      const float hx = gxt - sv.x, hy = gyt - sv.y;
      const float c = rho_scaled_f32(nu_code, __builtin_amdgcn_sqrtf(hx * hx + hy * hy));
      const __bf16 h = (__bf16)c;
      ah[j] = h;
      al[j] = (__bf16)(c - (float)h);
    }
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const int rr = 32 * b + (lane & 31);
      const bf16x8 bh = *reinterpret_cast<const bf16x8*>(Sh + rr * TK + kb);
      const bf16x8 bl = *reinterpret_cast<const bf16x8*>(Sl + rr * TK + kb);
      acc[b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh, acc[b], 0, 0, 0);
      acc[b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl, acc[b], 0, 0, 0);
      acc[b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh, acc[b], 0, 0, 0);
    }
    __syncthreads();
  }
  // accumulator layout of the 32x32 result: lane l, element e holds
  // row 8 (e / 4) + 4 (l / 32) + (e % 4) and column l % 32.
#pragma unroll
  for (int b = 0; b < 8; ++b)
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int gg = g0 + 32 * wave + 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3);
      const int r = r0 + 32 * b + (lane & 31);
      if (gg < M && r < R) fields[(size_t)r * M + gg] += acc[b][e];
    }
}

// ------------------------------------------------------------------- host

cesim_status chol_factor_device(cesim_ctx c, double tau2);
cesim_status chol_solve_device(cesim_ctx c, double* X, int R);
cesim_status lk_phi_device(cesim_ctx c, double tau2);
cesim_status lk_synth_rhs_device(cesim_ctx c, const void* fields, double* rhs);

// Linear map U (range units) and the per-path coordinate scale.
static void cov_map(const cesim_ctx c, double scale, double& ux, double& uxy, double& uyx,
                    double& uy) {
  ux = c->covd.u00 * scale;
  uxy = c->covd.u01 * scale;
  uyx = c->covd.u10 * scale;
  uy = c->covd.u11 * scale;
}

cesim_status condition_device(cesim_ctx c, double nugget, void* fields) {
  hipStream_t s = c->stream;
  const int n = c->nobs, R = c->nreal;
  if (!c->chol_valid || c->chol_nugget != nugget) {
    c->chol_valid = false;
    CESIM_TRY(chol_factor_device(c, nugget));
    c->chol_valid = true;
    c->chol_nugget = nugget;
  }
  CESIM_TRY(lk_phi_device(c, nugget));
  CESIM_TRY(c->coef.reserve(sizeof(double) * (size_t)n * R));
  double* X = c->coef.as<double>();
  CESIM_TRY(lk_synth_rhs_device(c, fields, X));
  CESIM_TRY(chol_solve_device(c, X, R));
  const int m1 = c->grid.m1, M = c->grid.m1 * c->grid.m2;
  const double dx = c->grid.dx, dy = c->grid.dy;
  if (c->prec == CESIM_PREC_FP64) {
    double ux, uxy, uyx, uy;
    cov_map(c, 1.0, ux, uxy, uyx, uy);
    dim3 grid((M + 127) / 128, (R + 63) / 64);
    const int tr = c->timer.begin(ST_KRIGE_GEMM, s);
    k_krige_f64<<<grid, 256, 0, s>>>(static_cast<double*>(fields), m1, M, R, X, n,
                                     c->obs_t64.as<double2>(), ux, uxy, uyx, uy, dx, dy,
                                     c->covd.nu_code, c->covd.sigma2);
    CESIM_HIP(hipGetLastError());
    c->timer.end(tr, s);
    return CESIM_OK;
  }
  const int Rp = (R + 255) / 256 * 256;
  const int npad = (n + 15) / 16 * 16;
  CESIM_TRY(c->coef_b16.reserve(sizeof(__bf16) * 2 * (size_t)npad * Rp));
  __bf16* Bh = c->coef_b16.as<__bf16>();
  __bf16* Bl = Bh + (size_t)npad * Rp;
  int tr = c->timer.begin(ST_COEF_SPLIT, s);
  k_split_coef<<<dim3((npad + 255) / 256, Rp), 256, 0, s>>>(X, n, R, Rp, c->covd.sigma2, Bh, Bl);
  CESIM_HIP(hipGetLastError());
  c->timer.end(tr, s);
  const double kappa = c->covd.nu_code == 0 ? kLog2e : (c->covd.nu_code == 2 ? kSqrt3 : kSqrt2);
  double ux, uxy, uyx, uy;
  cov_map(c, kappa, ux, uxy, uyx, uy);
  dim3 grid((M + 127) / 128, Rp / 256);
  tr = c->timer.begin(ST_KRIGE_GEMM, s);
  k_krige_bf16x3<<<grid, 256, 0, s>>>(static_cast<float*>(fields), m1, M, R, Rp, Bh, Bl, n,
                                      c->obs_t32.as<float2>(), (float)ux, (float)uxy, (float)uyx,
                                      (float)uy, (float)dx, (float)dy, c->covd.nu_code);
  CESIM_HIP(hipGetLastError());
  c->timer.end(tr, s);
  return CESIM_OK;
}

}  // namespace cesim
