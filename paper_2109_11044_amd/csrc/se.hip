// se.hip -- prediction standard errors on the grid, FP64 (Section 3, eq. (4);
// Section 3.1):
//   SE_E(g)^2 = C(0) - K12[g] A^{-1} K21[g],   A = K22 + tau^2 I,
//   SE_L(g)^2 = W2_g Q W2_g^T - 2 W2_g (W1 K11)[:, g] + C(0) + sum_i W2_gi^2 phi_i^2,
// the exact Kriging standard error and the one the local-Kriging simulation
// realizes (the diagonal of (Lambda - I) K11 (Lambda - I)^T + W2 diag(phi^2)
// W2^T with Lambda = W2 W1), where W2_g = K12[g] A^{-1}, Q = W1 K11 W1^T and
// phi_i^2 = tau^2 + gamma_i.  Grid nodes are processed in chunks of R: the
// cross-covariance rows K (R x n), X = W2 rows (the observation factor's
// solve with R right-hand sides), V = (W1 K11)^T rows (R x n, from a table
// of the covariance at grid lags), T = X Q (FP64 matrix-core GEMM), then one
// fixed-order reduction per node.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "internal.hpp"

namespace cesim {
namespace {

__device__ inline double node_x(const GridDev& g, int gg) {
  return __dadd_rn(g.x0, __dmul_rn((double)(gg % g.m1), g.dx));
}
__device__ inline double node_y(const GridDev& g, int gg) {
  return __dadd_rn(g.y0, __dmul_rn((double)(gg / g.m1), g.dy));
}

// K[r][i] = C(g_{g0 + r} - s_i); rows past the grid are zero.
__global__ void k_cross_chunk(const double* __restrict__ obs, int n, GridDev g, CovDev cov, int g0,
                              int R, int M, double* __restrict__ K) {
  const size_t q = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (q >= (size_t)R * n) return;
  const int r = (int)(q / n), i = (int)(q % n), gg = g0 + r;
  K[q] = gg < M ? cov_eval(cov, node_x(g, gg) - obs[2 * i], node_y(g, gg) - obs[2 * i + 1]) : 0.0;
}

// Covariance at every grid lag: T[(dy + m2 - 1)(2 m1 - 1) + dx + m1 - 1] =
// C(dx dx_grid, dy dy_grid) for |dx| < m1, |dy| < m2.  Window nodes and grid
// nodes differ by such lags, so the two products below read the table
// instead of evaluating the covariance.
__global__ void k_lag_table(GridDev g, CovDev cov, double* __restrict__ T) {
  const int w = 2 * g.m1 - 1;
  const size_t q = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (q >= (size_t)w * (2 * g.m2 - 1)) return;
  const int dx = (int)(q % w) - (g.m1 - 1), dy = (int)(q / w) - (g.m2 - 1);
  T[q] = cov_eval(cov, (double)dx * g.dx, (double)dy * g.dy);
}

// V[r][i] = sum_al w_i[al] C(node_{i,al} - g_{g0 + r}) = (W1 K11)[i][g] for a
// 64-node x 64-station tile: lane = node (consecutive nodes read consecutive
// table entries), each wave 16 stations, then an LDS transpose so that the
// stores run along the stations.  Nodes past the grid get zero rows.
template <int NPP>
__global__ void __launch_bounds__(256)
k_w1k_tab(const int2* __restrict__ corners, const double* __restrict__ W, int n, GridDev g,
          const double* __restrict__ T, int g0, int R, int M, double* __restrict__ V) {
  constexpr int W2 = 2 * NPP, K = W2 * W2;
  __shared__ double tile[64][65];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r0 = blockIdx.y * 64, i0 = blockIdx.x * 64;
  const int r = r0 + lane, gg = g0 + r;
  const bool live = r < R && gg < M;
  const int tw = 2 * g.m1 - 1;
  const int gx = live ? gg % g.m1 : 0, gy = live ? gg / g.m1 : 0;
  for (int j = 0; j < 16; ++j) {
    const int ii = wave * 16 + j, i = i0 + ii;
    double acc = 0.0;
    if (live && i < n) {
      const int2 ab = corners[i];
      const double* w = W + (size_t)i * K;
      const int base = (ab.y - gy + g.m2 - 1) * tw + ab.x - gx + g.m1 - 1;
#pragma unroll
      for (int q = 0; q < W2; ++q) {
        const double* t = T + base + q * tw;
#pragma unroll
        for (int p = 0; p < W2; ++p) acc += w[q * W2 + p] * t[p];
      }
    }
    tile[ii][lane] = acc;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < 64 * 64; e += 256) {
    const int rr = e >> 6, ii = e & 63;
    if (r0 + rr < R && i0 + ii < n) V[(size_t)(r0 + rr) * n + i0 + ii] = tile[ii][rr];
  }
}

// Q[i][j] = sum_al sum_be w_i[al] w_j[be] C(node_{i,al} - node_{j,be}).
template <int NPP>
__global__ void k_w1k11w1(const int2* __restrict__ corners, const double* __restrict__ W, int n,
                          GridDev g, const double* __restrict__ T, double* __restrict__ Q) {
  constexpr int W2 = 2 * NPP, K = W2 * W2;
  const size_t q = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (q >= (size_t)n * n) return;
  const int i = (int)(q / n), j = (int)(q % n);
  const int2 ai = corners[i], aj = corners[j];
  const double* wi = W + (size_t)i * K;
  const double* wj = W + (size_t)j * K;
  const int tw = 2 * g.m1 - 1;
  const int base = (ai.y - aj.y + g.m2 - 1) * tw + ai.x - aj.x + g.m1 - 1;
  double acc = 0.0;
  for (int al = 0; al < K; ++al) {
    const double* t = T + base + (al / W2) * tw + al % W2;
    double inner = 0.0;
    for (int be = 0; be < K; ++be) inner += wj[be] * t[-(be / W2) * tw - be % W2];
    acc += wi[al] * inner;
  }
  Q[q] = acc;
}

// One workgroup per node of the chunk: the four row products and the two
// standard errors.
__global__ void __launch_bounds__(256)
k_se_rows(const double* __restrict__ K, const double* __restrict__ X, const double* __restrict__ V,
          const double* __restrict__ T, const double* __restrict__ gam, double tau2, int n, int g0,
          int M, double sigma2, double* __restrict__ se_e, double* __restrict__ se_l) {
  __shared__ double red[4][256];
  const int r = blockIdx.x, gg = g0 + r;
  if (gg >= M) return;
  const size_t o = (size_t)r * n;
  double a = 0.0, b = 0.0, c = 0.0, d = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) {
    const double x = X[o + i];
    a += T[o + i] * x;
    b += x * V[o + i];
    c += x * x * (tau2 + gam[i]);
    d += x * K[o + i];
  }
  red[0][threadIdx.x] = a;
  red[1][threadIdx.x] = b;
  red[2][threadIdx.x] = c;
  red[3][threadIdx.x] = d;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h)
      for (int u = 0; u < 4; ++u) red[u][threadIdx.x] += red[u][threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    se_e[gg] = sqrt(fmax(0.0, sigma2 - red[3][0]));
    se_l[gg] = sqrt(fmax(0.0, red[0][0] - 2.0 * red[1][0] + sigma2 + red[2][0]));
  }
}

// X <- X A^{-1} for the R rows of X ([R][n]) by left-looking blocked
// substitutions with the observation factor L (amat) and its diagonal-block
// inverses W (winv): each block's update is one GEMM over every block solved
// before it (K up to n, N = one block), which keeps the GEMMs long in K for
// the many right-hand sides here.  Y: second R x n buffer.
//   forward block b:  X_b -= Y_{<b} L_{b,<b}^T;   Y_b = X_b W_b^T
//   backward block b: Y_b -= X_{>b} L_{>b,b};     X_b = Y_b W_b
cesim_status solve_rows_left(cesim_ctx c, double* X, double* Y, int R, hipStream_t s) {
  const int n = c->nobs, nbig = (n + kSolveBlock - 1) / kSolveBlock;
  const double* L = c->amat.as<double>();
  const double* Wi = c->winv.as<double>();
  const int tr = c->timer.begin(ST_SOLVE, s);
  for (int kb = 0; kb < nbig; ++kb) {
    const int K0 = kb * kSolveBlock, nb = std::min(kSolveBlock, n - K0);
    GemmArgs g;
    if (K0 > 0) {
      g.M = R; g.N = nb; g.K = K0; g.alpha = -1.0; g.beta = 1.0;
      g.A = Y; g.sai = n; g.sak = 1;
      g.B = L + (size_t)K0 * n; g.sbk = 1; g.sbj = n;      // B(t, c) = L[K0 + c][t]
      g.C = X + K0; g.sci = n; g.scj = 1;
      CESIM_TRY(gemm_f64(g, false, s));
    }
    g.M = R; g.N = nb; g.K = nb; g.alpha = 1.0; g.beta = 0.0;
    g.A = X + K0; g.sai = n; g.sak = 1;
    g.B = Wi + (size_t)kb * kSolveBlock * kSolveBlock; g.sbk = 1; g.sbj = kSolveBlock;
    g.C = Y + K0; g.sci = n; g.scj = 1;
    CESIM_TRY(gemm_f64(g, false, s));
  }
  for (int kb = nbig - 1; kb >= 0; --kb) {
    const int K0 = kb * kSolveBlock, nb = std::min(kSolveBlock, n - K0), rest = n - K0 - nb;
    GemmArgs g;
    if (rest > 0) {
      g.M = R; g.N = nb; g.K = rest; g.alpha = -1.0; g.beta = 1.0;
      g.A = X + K0 + nb; g.sai = n; g.sak = 1;
      g.B = L + (size_t)(K0 + nb) * n + K0; g.sbk = n; g.sbj = 1;   // B(t, i) = L[K0+nb+t][K0+i]
      g.C = Y + K0; g.sci = n; g.scj = 1;
      CESIM_TRY(gemm_f64(g, false, s));
    }
    g.M = R; g.N = nb; g.K = nb; g.alpha = 1.0; g.beta = 0.0;
    g.A = Y + K0; g.sai = n; g.sak = 1;
    g.B = Wi + (size_t)kb * kSolveBlock * kSolveBlock; g.sbk = kSolveBlock; g.sbj = 1;
    g.C = X + K0; g.sci = n; g.scj = 1;
    CESIM_TRY(gemm_f64(g, false, s));
  }
  c->timer.end(tr, s);
  return CESIM_OK;
}

// at most 65535 tiles of 64 nodes along the second grid dimension
constexpr int kMaxChunk = 65535 * 64;

}  // namespace
}  // namespace cesim

using namespace cesim;

extern "C" cesim_status ce_prediction_se(cesim_ctx c, double nugget, void* se_exact,
                                         void* se_local) {
  if (!c || !se_exact || !se_local) return CESIM_ERR_INVALID_ARG;
  if (!(std::isfinite(nugget) && nugget >= 0.0)) return CESIM_ERR_INVALID_ARG;
  if (c->nobs < 1) return CESIM_ERR_BAD_STATE;
  if (joint_active(c)) return CESIM_ERR_INVALID_ARG;   // the closed form is of independent sampling
  hipStream_t s = c->stream;
  CESIM_HIP(hipStreamSynchronize(c->aux));       // earlier aux work may use the factor
  CESIM_HIP(hipStreamSynchronize(s));
  const int n = c->nobs, M = c->grid.m1 * c->grid.m2;
  // chunk of grid nodes: five R x n arrays within about 16 GiB unless set
  // (larger chunks keep the substitution GEMMs' grids full)
  const size_t per_row = 5 * (size_t)n * sizeof(double);
  const int R = std::min(kMaxChunk, c->se_chunk > 0 ? std::min(c->se_chunk, M)
                                  : (int)std::max<size_t>(64, std::min<size_t>(
                                        (size_t)M, ((size_t)16 << 30) / per_row)));
  const size_t nlag = (size_t)(2 * c->grid.m1 - 1) * (2 * c->grid.m2 - 1);
  CESIM_TRY(c->sework.reserve(per_row * R + sizeof(double) * ((size_t)n * n + nlag)));
  double* K = c->sework.as<double>();
  double* X = K + (size_t)R * n;
  double* Y = X + (size_t)R * n;
  double* V = Y + (size_t)R * n;
  double* T = V + (size_t)R * n;
  double* Q = T + (size_t)R * n;
  double* lag = Q + (size_t)n * n;
  const bool refactor = !c->chol_valid || c->chol_nugget != nugget;
  if (refactor) {
    c->chol_valid = false;
    CESIM_TRY(chol_factor_device(c, nugget, s));
  }
  const double* obs = c->obs_xy.as<double>();
  const int2* cor = c->corners.as<int2>();
  const double* W = c->weights.as<double>();
  const unsigned nq = (unsigned)(((size_t)n * n + 255) / 256);
#define CESIM_NP(NP, CALL) \
  case NP: CALL; break;
  int tr = c->timer.begin(ST_SE_Q, s);
  k_lag_table<<<(unsigned)((nlag + 255) / 256), 256, 0, s>>>(c->gridd, c->covd, lag);
  CESIM_HIP(hipGetLastError());
  switch (c->npp) {
    CESIM_NP(1, (k_w1k11w1<1><<<nq, 256, 0, s>>>(cor, W, n, c->gridd, lag, Q)))
    CESIM_NP(2, (k_w1k11w1<2><<<nq, 256, 0, s>>>(cor, W, n, c->gridd, lag, Q)))
    CESIM_NP(3, (k_w1k11w1<3><<<nq, 256, 0, s>>>(cor, W, n, c->gridd, lag, Q)))
    default: k_w1k11w1<4><<<nq, 256, 0, s>>>(cor, W, n, c->gridd, lag, Q); break;
  }
  CESIM_HIP(hipGetLastError());
  c->timer.end(tr, s);
  const unsigned nr = (unsigned)(((size_t)R * n + 255) / 256);
  const dim3 tiles((unsigned)((n + 63) / 64), (unsigned)((R + 63) / 64));
  for (int g0 = 0; g0 < M; g0 += R) {
    tr = c->timer.begin(ST_SE_COV_ROWS, s);
    k_cross_chunk<<<nr, 256, 0, s>>>(obs, n, c->gridd, c->covd, g0, R, M, K);
    CESIM_HIP(hipGetLastError());
    switch (c->npp) {
      CESIM_NP(1, (k_w1k_tab<1><<<tiles, 256, 0, s>>>(cor, W, n, c->gridd, lag, g0, R, M, V)))
      CESIM_NP(2, (k_w1k_tab<2><<<tiles, 256, 0, s>>>(cor, W, n, c->gridd, lag, g0, R, M, V)))
      CESIM_NP(3, (k_w1k_tab<3><<<tiles, 256, 0, s>>>(cor, W, n, c->gridd, lag, g0, R, M, V)))
      default: k_w1k_tab<4><<<tiles, 256, 0, s>>>(cor, W, n, c->gridd, lag, g0, R, M, V); break;
    }
    CESIM_HIP(hipGetLastError());
    c->timer.end(tr, s);
    CESIM_HIP(hipMemcpyAsync(X, K, sizeof(double) * (size_t)R * n, hipMemcpyDeviceToDevice, s));
    CESIM_TRY(solve_rows_left(c, X, Y, R, s));                // X = K A^{-1} (rows of W2)
    GemmArgs gm;                                               // T = X Q
    gm.M = R; gm.N = n; gm.K = n; gm.alpha = 1.0; gm.beta = 0.0;
    gm.A = X; gm.sai = n; gm.sak = 1;
    gm.B = Q; gm.sbk = n; gm.sbj = 1;
    gm.C = T; gm.sci = n; gm.scj = 1;
    tr = c->timer.begin(ST_SE_GEMM, s);
    CESIM_TRY(gemm_f64(gm, false, s));
    c->timer.end(tr, s);
    tr = c->timer.begin(ST_SE_REDUCE, s);
    k_se_rows<<<std::min(R, M - g0), 256, 0, s>>>(K, X, V, T, c->gamma.as<double>(), nugget, n, g0,
                                                   M, c->covd.sigma2,
                                                   static_cast<double*>(se_exact),
                                                   static_cast<double*>(se_local));
    CESIM_HIP(hipGetLastError());
    c->timer.end(tr, s);
  }
#undef CESIM_NP
  CESIM_HIP(hipStreamSynchronize(s));
  if (refactor) {
    if (c->chol_info_host[0] & 2) return CESIM_ERR_NOT_POSITIVE_DEFINITE;
    c->chol_valid = true;
    c->chol_nugget = nugget;
  }
  return CESIM_OK;
}
