// linalg.hip -- FP64 Kriging system of the observations (eq. (4), Section 3;
// steps 1 and 4 of Section 2):
//   A = K22 + tau^2 I,  A = L L^T (blocked right-looking Cholesky),
//   X = A^{-1} RHS for all realizations (blocked forward and backward
//   substitution with the inverses of the diagonal blocks).
// Besides the diagonal-block factorisation, every step (panel solves,
// trailing updates, diagonal-block applications, solve updates) is one call
// of the FP64 matrix-core GEMM below.
// The O(n^3) trailing updates and O(n^2 R) solve updates run in one generic
// FP64 matrix-core GEMM (v_mfma_f64_16x16x4f64, 64 x 64 or 32 x 32 tiles).
#include <hip/hip_runtime.h>

#include <cstring>
#include <vector>

#include "internal.hpp"

namespace cesim {

typedef double doublex4 __attribute__((ext_vector_type(4)));

constexpr int kNB = 64;   // Cholesky block size
constexpr int kSB = kSolveBlock;  // substitution block size (4 Cholesky blocks)
constexpr long kSmallGemmTiles = 320;   // fewer 64 x 64 tiles than this: 32 x 32 tiles

// A = K22 + tau^2 I (+ diag(extra) for the surrogate sites of
// nearest-neighbour Kriging, whose nugget is inflated site by site).
__global__ void k_assemble_a(const double* __restrict__ obs, int n, CovDev cov, double tau2,
                             const double* __restrict__ extra, double* __restrict__ A) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y;
  if (j >= n) return;
  double v = cov_eval(cov, obs[2 * i] - obs[2 * j], obs[2 * i + 1] - obs[2 * j + 1]);
  if (i == j) v += extra ? tau2 + extra[i] : tau2;
  A[(size_t)i * n + j] = v;
}

// The factorisation and the substitutions are chains of small dependent
// kernels that share the CUs with throughput kernels running beside them
// (the draw, the prediction).  Their waves take the highest issue priority
// on their SIMD, so that the chain is not slowed by the waves it shares the
// SIMD with; the throughput kernels fill the cycles it leaves.
__device__ __forceinline__ void chain_priority() { __builtin_amdgcn_s_setprio(3); }

// Copies the inverse of each 64 x 64 diagonal factor block kb into its
// place in the 256 x 256 block inverse W[kb / 4] (zeroed beforehand).
__global__ void __launch_bounds__(256)
k_place_diag(const double* __restrict__ D, int n, double* __restrict__ W) {
  chain_priority();
  const int kb = blockIdx.x, big = kb / 4, i = kb % 4;
  const int sz = min(kNB, n - kb * kNB);
  double* w = W + (size_t)big * kSB * kSB + (size_t)(kNB * i) * kSB + kNB * i;
  const double* d = D + (size_t)kb * kNB * kNB;
  for (int e = threadIdx.x; e < kNB * kNB; e += 256) {
    const int a = e / kNB, cc = e % kNB;
    if (a < sz && cc < sz) w[(size_t)a * kSB + cc] = d[e];
  }
}

// Lane l's value of v (l uniform): two 32-bit lane reads into scalar
// registers, which the next instruction takes as an operand.
__device__ __forceinline__ double lane_value(double v, int l) {
  const long long u = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)u, l);
  const int hi = __builtin_amdgcn_readlane((int)(u >> 32), l);
  return __hiloint2double(hi, lo);
}

// Factor the nbk x nbk diagonal block at (k0, k0) and form the inverse of
// its factor; 256 threads.  Wave 0 factors: lane i holds row i in registers
// (every index static, the loops unrolled) and, right-looking, at pivot j
// reads the pivot and the unscaled column-j entries of the rows k > j from
// their lanes and updates its row.  The inverse X = L^{-1} is then formed
// by rows with all four waves: at step k row k of X is final, X[k][c] =
// x_k[c] / L[k][k], and every row i > k subtracts L[i][k] X[k][c]; wave w
// holds the columns c = 4 m + w of row i in lane i and reads L from LDS.
// Each entry of X is the same sum in the same order as by forward
// substitution on the columns of the identity.  Writes L back (lower part)
// and the inverse to dinv (kNB x kNB, row-major, zero above the diagonal,
// the identity past nbk); bit 2 of *info marks a non-positive pivot.
__device__ __forceinline__ void potrf_diag_body(double* __restrict__ A, int n, int k0, int nbk,
                                                double* __restrict__ dinv, int* __restrict__ info) {
  // L packed by columns (column k holds rows k..63 from kcol(k)): 16.6 KB,
  // small enough to share a CU with the draw kernels when condition()
  // overlaps them
  __shared__ double Lc[kNB * (kNB + 1) / 2];
  __shared__ double rinv[kNB];          // 1 / L[i][i]
  auto kcol = [](int k) { return k * kNB - k * (k - 1) / 2; };
  const int t = threadIdx.x, i = t & 63;
  if (t < 64) {
    double a[kNB];
    bool bad = false;
#pragma unroll
    for (int k = 0; k < kNB; ++k)
      a[k] = (i < nbk && k < nbk) ? A[(size_t)(k0 + i) * n + k0 + k] : (i == k ? 1.0 : 0.0);
    double myinv = 0.0;
#pragma unroll
    for (int j = 0; j < kNB; ++j) {
      const double cj = a[j];               // column j of row i, not yet scaled
      const double d = lane_value(cj, j);
      bad |= (j < nbk && !(d > 0.0));
      const double piv = sqrt(d), r = 1.0 / piv;
      a[j] = (i > j) ? cj * r : (i == j ? piv : 0.0);
      const double lij = a[j] * r;          // L[i][j] / L[j][j]: pairs with unscaled entries
      if (i == j) myinv = r;
#pragma unroll
      for (int k = j + 1; k < kNB; ++k)     // entries k > i of row i are never read
        a[k] = fma(-lij, lane_value(cj, k), a[k]);
    }
#pragma unroll
    for (int k = 0; k < kNB; ++k) {
      if (k <= i) Lc[kcol(k) + i - k] = a[k];
      if (i < nbk && k <= i) A[(size_t)(k0 + i) * n + k0 + k] = a[k];
    }
    rinv[i] = myinv;
    if (bad && i == 0) atomicOr(info, 2);
  }
  __syncthreads();
  const int w = __builtin_amdgcn_readfirstlane(t >> 6);
  double x[kNB / 4];
#pragma unroll
  for (int m = 0; m < kNB / 4; ++m) x[m] = (4 * m + w == i) ? 1.0 : 0.0;
  for (int k = 0; k < kNB; ++k) {
    const double lik = (i > k) ? Lc[kcol(k) + i - k] : 0.0;
    const double rk = rinv[k];
    // columns c > k of row k are zero and leave x unchanged
#pragma unroll
    for (int m = 0; m < kNB / 4; ++m) x[m] = fma(-lik, lane_value(x[m], k) * rk, x[m]);
  }
  const double ri = rinv[i];
#pragma unroll
  for (int m = 0; m < kNB / 4; ++m) {
    const int c = 4 * m + w;
    dinv[i * kNB + c] = (c <= i) ? x[m] * ri : 0.0;
  }
}

__global__ void __launch_bounds__(256)
k_potrf_diag(double* __restrict__ A, int n, int k0, int nbk, double* __restrict__ dinv,
             int* __restrict__ info) {
  chain_priority();
  potrf_diag_body(A, n, k0, nbk, dinv, info);
}

// One diagonal block of each of several systems: workgroup q takes d[q].
__global__ void __launch_bounds__(256) k_potrf_diag_grp(const DiagDesc* __restrict__ d) {
  chain_priority();
  const DiagDesc e = d[blockIdx.x];
  potrf_diag_body(e.A, e.n, e.k0, e.nbk, e.dinv, e.info);
}

// Generic FP64 GEMM on matrix cores (GemmArgs): T x T tiles (T = 64 or 32),
// 4 waves of T/2 x T/2, k-step 16.  LOWER: skip tiles strictly above the
// diagonal (symmetric updates).  Both tile sizes sum every output element
// in the same order (k-steps of 4 in ascending order), so the choice of T
// never changes a result.
// Operand layouts of v_mfma_f64_16x16x4f64: lane l holds A[l % 16][l / 16]
// and B[l / 16][l % 16]; accumulator v of lane l is D[l / 16 + 4 v][l % 16].
template <int T, bool LOWER>
__device__ __forceinline__ void f64_tile(const GemmArgs& g, int bi, int bj) {
  constexpr int TK = 16, WT = T / 2, FB = WT / 16;   // FB x FB blocks of 16 x 16 per wave
  constexpr int NE = T * TK / 256;                   // operand elements per thread and k-step
  __shared__ double As[2][TK][T + 2];
  __shared__ double Bs[2][TK][T + 2];
  if (LOWER && bj > bi) return;
  const int i0 = bi * T, j0 = bj * T;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wr = (wave >> 1) * WT, wc = (wave & 1) * WT;
  doublex4 acc[FB][FB];
#pragma unroll
  for (int a = 0; a < FB; ++a)
#pragma unroll
    for (int b = 0; b < FB; ++b) acc[a][b] = (doublex4){0.0, 0.0, 0.0, 0.0};
  const bool a_ifast = (g.sai == 1);
  const bool b_jfast = (g.sbj == 1);
  // element u of this thread's share of a k-step: (row, k) of the A tile
  // and (k, column) of the B tile, along the operand's contiguous index
  int ai[NE], ak[NE], bj_[NE], bk[NE];
#pragma unroll
  for (int u = 0; u < NE; ++u) {
    const int e = threadIdx.x + 256 * u;
    if (a_ifast) { ai[u] = e % T; ak[u] = e / T; } else { ak[u] = e % TK; ai[u] = e / TK; }
    if (b_jfast) { bj_[u] = e % T; bk[u] = e / T; } else { bk[u] = e % TK; bj_[u] = e / TK; }
  }
  double ra[NE], rb[NE];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int u = 0; u < NE; ++u) {
      const int gi = i0 + ai[u], gk = k0 + ak[u];
      ra[u] = (gi < g.M && gk < g.K) ? g.A[gi * g.sai + gk * g.sak] : 0.0;
      const int gj = j0 + bj_[u], gk2 = k0 + bk[u];
      rb[u] = (gj < g.N && gk2 < g.K) ? g.B[gk2 * g.sbk + gj * g.sbj] : 0.0;
    }
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int u = 0; u < NE; ++u) {
      As[buf][ak[u]][ai[u]] = ra[u];
      Bs[buf][bk[u]][bj_[u]] = rb[u];
    }
  };
  // one barrier per k-step: the next step's operands are fetched into
  // registers during this step's products and stored into the other buffer
  fetch(0);
  stash(0);
  __syncthreads();
  int buf = 0;
  for (int k0 = 0; k0 < g.K; k0 += TK) {
    const bool more = k0 + TK < g.K;
    if (more) fetch(k0 + TK);
#pragma unroll
    for (int ks = 0; ks < TK; ks += 4) {
      const int kk = ks + (lane >> 4);
      double a[FB], b[FB];
#pragma unroll
      for (int t = 0; t < FB; ++t) {
        a[t] = As[buf][kk][wr + 16 * t + (lane & 15)];
        b[t] = Bs[buf][kk][wc + 16 * t + (lane & 15)];
      }
#pragma unroll
      for (int x = 0; x < FB; ++x)
#pragma unroll
        for (int y = 0; y < FB; ++y)
          acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[x], b[y], acc[x][y], 0, 0, 0);
    }
    if (more) stash(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
#pragma unroll
  for (int x = 0; x < FB; ++x)
#pragma unroll
    for (int y = 0; y < FB; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int gi = i0 + wr + 16 * x + (lane >> 4) + 4 * v;
        const int gj = j0 + wc + 16 * y + (lane & 15);
        if (gi < g.M && gj < g.N) {
          double* cp = g.C + gi * g.sci + gj * g.scj;
          const double prev = g.beta != 0.0 ? *cp : 0.0;
          *cp = g.alpha * acc[x][y][v] + g.beta * prev;
        }
      }
}

template <int T, bool LOWER>
__global__ void __launch_bounds__(256) k_gemm_f64(GemmArgs g) {
  chain_priority();
  f64_tile<T, LOWER>(g, blockIdx.y, blockIdx.x);
}

// Several independent GEMMs in one launch: group q owns workgroups
// [tile0[q], tile0[q + 1]) (ascending, no empty groups), its tiles in
// row-major order of its 64 x 64 tile grid.
template <bool LOWER>
__global__ void __launch_bounds__(256)
k_gemm_f64_grp(const GemmArgs* __restrict__ gs, const int* __restrict__ tile0, int ngroups) {
  chain_priority();
  const int b = blockIdx.x;
  int lo = 0, hi = ngroups - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (tile0[mid] <= b) lo = mid;
    else hi = mid - 1;
  }
  const GemmArgs g = gs[lo];
  const int t = b - tile0[lo];
  const int tn = (g.N + 63) / 64;
  f64_tile<64, LOWER>(g, t / tn, t % tn);
}

// 64 x 64 tiles, or 32 x 32 where 64 x 64 tiles would leave most CUs idle
// (the diagonal-block applications of the substitutions, the column
// updates of the factorisation): four times the workgroups at half the
// operand reuse.  An in-place product (rows_in_place) keeps one workgroup
// per row block.
cesim_status gemm_f64(const GemmArgs& g, bool lower, hipStream_t s, bool rows_in_place) {
  if (g.M <= 0 || g.N <= 0 || g.K <= 0) return CESIM_OK;
  if (rows_in_place && g.N > 64) return CESIM_ERR_INVALID_ARG;
  const long tiles64 = (long)((g.N + 63) / 64) * ((g.M + 63) / 64);
  if (tiles64 < kSmallGemmTiles && !rows_in_place) {
    dim3 grid((g.N + 31) / 32, (g.M + 31) / 32);
    if (lower) k_gemm_f64<32, true><<<grid, 256, 0, s>>>(g);
    else k_gemm_f64<32, false><<<grid, 256, 0, s>>>(g);
  } else {
    dim3 grid((g.N + 63) / 64, (g.M + 63) / 64);
    if (lower) k_gemm_f64<64, true><<<grid, 256, 0, s>>>(g);
    else k_gemm_f64<64, false><<<grid, 256, 0, s>>>(g);
  }
  CESIM_HIP(hipGetLastError());
  return CESIM_OK;
}

// Inverses W_B of the 256 x 256 diagonal blocks of the factor of every
// context, for the substitutions.  With the 64-block inverses D_i on its
// diagonal, block row i of W_B is W_{i,0:i} = -D_i (L_{i,0:i} W_{0:i,0:i})
// (block forward substitution on the identity); rows i = 1, 2, 3 in turn,
// each as two grouped GEMMs over all blocks of all contexts.  With keep
// (one context) the launch table is uploaded through the context's pinned
// stage and kept there, and nothing synchronises; otherwise synchronises.
static cesim_status build_winv(const std::vector<cesim_ctx>& cs, hipStream_t s,
                               GroupedSeq* keep = nullptr) {
  std::vector<std::vector<GemmArgs>> lv(6);
  for (cesim_ctx c : cs) {
    const int n = c->nobs, nblk = (n + kNB - 1) / kNB, nbig = (n + kSB - 1) / kSB;
    CESIM_TRY(c->winv.reserve(sizeof(double) * (size_t)nbig * kSB * kSB));
    CESIM_TRY(c->wtmp.reserve(sizeof(double) * (size_t)nbig * kNB * (kSB - kNB)));
    double* W = c->winv.as<double>();
    CESIM_HIP(hipMemsetAsync(W, 0, sizeof(double) * (size_t)nbig * kSB * kSB, s));
    k_place_diag<<<nblk, 256, 0, s>>>(c->dinv.as<double>(), n, W);
    CESIM_HIP(hipGetLastError());
    const double* L = c->amat.as<double>();
    const double* D = c->dinv.as<double>();
    for (int B = 0; B < nbig; ++B) {
      const int K0 = B * kSB, nb = std::min(kSB, n - K0);
      double* WB = W + (size_t)B * kSB * kSB;
      double* TB = c->wtmp.as<double>() + (size_t)B * kNB * (kSB - kNB);
      for (int i = 1; i * kNB < nb; ++i) {
        const int si = std::min(kNB, nb - kNB * i);
        GemmArgs g;        // T = L_{i,0:i} W_{0:i,0:i}
        g.M = si; g.N = kNB * i; g.K = kNB * i; g.alpha = 1.0; g.beta = 0.0;
        g.A = L + (size_t)(K0 + kNB * i) * n + K0; g.sai = n; g.sak = 1;
        g.B = WB; g.sbk = kSB; g.sbj = 1;
        g.C = TB; g.sci = kSB - kNB; g.scj = 1;
        lv[2 * (i - 1)].push_back(g);
        g.M = si; g.N = kNB * i; g.K = si; g.alpha = -1.0; g.beta = 0.0;   // W_{i,0:i} = -D_i T
        g.A = D + (size_t)(4 * B + i) * kNB * kNB; g.sai = kNB; g.sak = 1;
        g.B = TB; g.sbk = kSB - kNB; g.sbj = 1;
        g.C = WB + (size_t)(kNB * i) * kSB; g.sci = kSB; g.scj = 1;
        lv[2 * (i - 1) + 1].push_back(g);
      }
    }
  }
  if (keep) {
    keep->clear();
    keep->dev.stream = s;
    for (auto& v : lv) keep->add_gemm(v, false);
    if (keep->launches.empty()) return CESIM_OK;
    CESIM_TRY(keep->upload_async(s, cs[0]->winv_stage));
    return keep->launch(s);
  }
  GroupedSeq seq;
  for (auto& v : lv) seq.add_gemm(v, false);
  if (!seq.launches.empty()) {
    CESIM_TRY(seq.upload(s));
    CESIM_TRY(seq.launch(s));
    CESIM_HIP(hipStreamSynchronize(s));
    seq.dev.release();
  }
  return CESIM_OK;
}

// Factor A = K22 + tau^2 I in place (lower triangle) and build the block
// inverses of the solves, all queued on s without synchronising.  A
// non-positive pivot sets bit 2 of c->chol_info[0] on the device; its
// pinned copy c->chol_info_host is valid once work queued on s after this
// call has completed.  clear_info = false keeps flags set by work queued
// before on s (the box factors of the joint sampling).
cesim_status chol_factor_device(cesim_ctx c, double tau2, hipStream_t s, bool clear_info) {
  c->yhat_valid = false;
  c->ainv_valid = false;
  const int n = c->nobs;
  const int nblk = (n + kNB - 1) / kNB;
  CESIM_TRY(c->amat.reserve(sizeof(double) * (size_t)n * n));
  CESIM_TRY(c->dinv.reserve(sizeof(double) * (size_t)nblk * kNB * kNB));
  double* A = c->amat.as<double>();
  double* D = c->dinv.as<double>();
  int* info = c->chol_info.as<int>();
  if (clear_info) CESIM_HIP(hipMemsetAsync(info, 0, sizeof(int) * 4, s));
  const int tr = c->timer.begin(ST_CHOL, s);
  k_assemble_a<<<dim3((n + 255) / 256, n), 256, 0, s>>>(
      c->obs_xy.as<double>(), n, c->covd, tau2, c->nn_active ? c->nn_extra.as<double>() : nullptr,
      A);
  CESIM_HIP(hipGetLastError());
  // Right-looking, with look-ahead: after the panel of block kb, s updates
  // block column kb+1 alone and goes on to factor it, while the look stream
  // applies the rest of block kb's trailing update (the columns from kb+2
  // on).  The 64 x 64 tiles and each element's products are those of one
  // lower-triangular trailing update per block, so the factor is the same.
  hipStream_t la = c->look;
  bool la_pending = false;            // la_update marks look work s has not joined
  for (int kb = 0; kb < nblk; ++kb) {
    const int k0 = kb * kNB, nbk = std::min(kNB, n - k0);
    k_potrf_diag<<<1, 256, 0, s>>>(A, n, k0, nbk, D + (size_t)kb * kNB * kNB, info);
    CESIM_HIP(hipGetLastError());
    const int rest = n - k0 - nbk;
    if (rest <= 0) break;
    {   // panel: A[i, k0:k0+nbk] <- A[i, k0:k0+nbk] Linv^T (in place: each
        // workgroup reads its whole row block before writing it)
      GemmArgs g;
      g.M = rest; g.N = nbk; g.K = nbk; g.alpha = 1.0; g.beta = 0.0;
      g.A = A + (size_t)(k0 + nbk) * n + k0; g.sai = n; g.sak = 1;
      g.B = D + (size_t)kb * kNB * kNB; g.sbk = 1; g.sbj = kNB;     // B(t, c) = Linv[c][t]
      g.C = A + (size_t)(k0 + nbk) * n + k0; g.sci = n; g.scj = 1;
      CESIM_TRY(gemm_f64(g, false, s, true));
    }
    // trailing update A[i][j] -= sum_t P[i][t] P[j][t] (P: the panel) of
    // the rows and columns from c0, on the tiles of the lower triangle
    const int k1 = k0 + nbk;
    auto update = [&](int c0, int ncols, bool lower, hipStream_t st) {
      GemmArgs g;
      g.M = n - c0; g.N = ncols; g.K = nbk; g.alpha = -1.0; g.beta = 1.0;
      g.A = A + (size_t)c0 * n + k0; g.sai = n; g.sak = 1;
      g.B = A + (size_t)c0 * n + k0; g.sbk = 1; g.sbj = n;
      g.C = A + (size_t)c0 * n + c0; g.sci = n; g.scj = 1;
      return gemm_f64(g, lower, st);
    };
    const int nb1 = std::min(kNB, rest), rest2 = rest - nb1;
    if (!la || rest2 <= 0) {
      if (la_pending) CESIM_HIP(hipStreamWaitEvent(s, c->la_update, 0));
      la_pending = false;
      CESIM_TRY(update(k1, rest, true, s));
      continue;
    }
    // block column kb+1 (all its rows): the look stream's update of the
    // previous step wrote it too
    if (la_pending) CESIM_HIP(hipStreamWaitEvent(s, c->la_update, 0));
    {
      GemmArgs g;
      g.M = rest; g.N = nb1; g.K = nbk; g.alpha = -1.0; g.beta = 1.0;
      g.A = A + (size_t)k1 * n + k0; g.sai = n; g.sak = 1;
      g.B = A + (size_t)k1 * n + k0; g.sbk = 1; g.sbj = n;
      g.C = A + (size_t)k1 * n + k1; g.sci = n; g.scj = 1;
      CESIM_TRY(gemm_f64(g, false, s));
    }
    CESIM_HIP(hipEventRecord(c->la_panel, s));
    CESIM_HIP(hipStreamWaitEvent(la, c->la_panel, 0));
    CESIM_TRY(update(k1 + nb1, rest2, true, la));
    CESIM_HIP(hipEventRecord(c->la_update, la));
    la_pending = true;
  }
  if (la_pending) CESIM_HIP(hipStreamWaitEvent(s, c->la_update, 0));
  CESIM_HIP(hipMemcpyAsync(c->chol_info_host, info, sizeof(int) * 4, hipMemcpyDeviceToHost, s));
  // after a failed pivot the inverses are built from meaningless values;
  // nothing downstream writes the fields then
  CESIM_TRY(build_winv({c}, s, &c->winv_seq));
  c->timer.end(tr, s);
  return CESIM_OK;
}

// The GEMMs of the forward (L Y = X) and backward (L^T Z = Y) blocked
// substitutions of one system, in order, with 256-wide blocks and their
// inverses W (winv), as C(r, i) over realizations r (X, Y: [R][n]):
//   forward block kb:  Y[r][K0+c]    = sum_t X[r][K0+t] W[c][t]
//                      X[r][K0+nb+i] -= sum_t Y[r][K0+t] L[K0+nb+i][K0+t]
//   backward block kb: X[r][K0+c]    = sum_t Y[r][K0+t] W[t][c]
//                      Y[r][i]       -= sum_t X[r][K0+t] L[K0+t][i]   (i < K0)
// X holds the right-hand sides and ends with the solution; no GEMM writes
// what it reads.  Forward step kb is fwd[kb], backward step st (counted from
// the last block) bwd[st].
// identity: X = I (R = n) and Y zero on entry; row r of the forward
// solution L^{-1} e_r is zero before entry r, so forward block kb touches
// only rows r < K0 + nb (a third of the forward GEMMs' work).
static void solve_step_lists(cesim_ctx c, double* X, double* Y, int R,
                             std::vector<std::vector<GemmArgs>>& fwd,
                             std::vector<std::vector<GemmArgs>>& bwd, bool identity = false) {
  const int n = c->nobs, nbig = (n + kSB - 1) / kSB;
  const double* L = c->amat.as<double>();
  const double* W = c->winv.as<double>();
  fwd.assign(nbig, {});
  bwd.assign(nbig, {});
  for (int kb = 0; kb < nbig; ++kb) {
    const int K0 = kb * kSB, nb = std::min(kSB, n - K0), rest = n - K0 - nb;
    const double* WB = W + (size_t)kb * kSB * kSB;
    const int rows = identity ? std::min(R, K0 + nb) : R;
    GemmArgs g;
    g.M = rows; g.N = nb; g.K = nb; g.alpha = 1.0; g.beta = 0.0;
    g.A = X + K0; g.sai = n; g.sak = 1;
    g.B = WB; g.sbk = 1; g.sbj = kSB;
    g.C = Y + K0; g.sci = n; g.scj = 1;
    fwd[kb].push_back(g);
    if (rest > 0) {
      g.M = rows; g.N = rest; g.K = nb; g.alpha = -1.0; g.beta = 1.0;
      g.A = Y + K0; g.sai = n; g.sak = 1;
      g.B = L + (size_t)(K0 + nb) * n + K0; g.sbk = 1; g.sbj = n;
      g.C = X + K0 + nb; g.sci = n; g.scj = 1;
      fwd[kb].push_back(g);
    }
  }
  for (int st = 0; st < nbig; ++st) {
    const int kb = nbig - 1 - st, K0 = kb * kSB, nb = std::min(kSB, n - K0);
    const double* WB = W + (size_t)kb * kSB * kSB;
    GemmArgs g;
    g.M = R; g.N = nb; g.K = nb; g.alpha = 1.0; g.beta = 0.0;
    g.A = Y + K0; g.sai = n; g.sak = 1;
    g.B = WB; g.sbk = kSB; g.sbj = 1;
    g.C = X + K0; g.sci = n; g.scj = 1;
    bwd[st].push_back(g);
    if (K0 > 0) {
      g.M = R; g.N = K0; g.K = nb; g.alpha = -1.0; g.beta = 1.0;
      g.A = X + K0; g.sai = n; g.sak = 1;
      g.B = L + (size_t)K0 * n; g.sbk = n; g.sbj = 1;
      g.C = Y; g.sci = n; g.scj = 1;
      bwd[st].push_back(g);
    }
  }
}

static void solve_steps(cesim_ctx c, double* X, double* Y, int R, std::vector<GemmArgs>& out,
                        bool identity = false) {
  std::vector<std::vector<GemmArgs>> fwd, bwd;
  solve_step_lists(c, X, Y, R, fwd, bwd, identity);
  for (auto& v : fwd) out.insert(out.end(), v.begin(), v.end());
  for (auto& v : bwd) out.insert(out.end(), v.begin(), v.end());
}

// X[r][.] <- A^{-1} X[r][.] for r < R with the factor held in c->amat.
// Every step is a GEMM with the realizations as its rows, so that each lane
// of a tile writes consecutive observations of one realization (X is
// [R][n], observation index fastest).
// Y: second buffer of at least R n doubles; stage: the timer stage it counts in.
cesim_status chol_solve_device(cesim_ctx c, double* X, int R, hipStream_t s, double* Y,
                               int stage, bool identity) {
  const int tr = c->timer.begin(stage, s);
  std::vector<GemmArgs> steps;
  solve_steps(c, X, Y, R, steps, identity);
  for (const GemmArgs& g : steps) CESIM_TRY(gemm_f64(g, false, s));
  c->timer.end(tr, s);
  return CESIM_OK;
}

// --------------------------------------------------------- explicit inverse

// X = I and Y = 0 (n x n each).
__global__ void __launch_bounds__(256) k_identity(double* __restrict__ X, double* __restrict__ Y,
                                                  int n) {
  const size_t q = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (q < (size_t)n * n) {
    X[q] = (q / n == q % n) ? 1.0 : 0.0;
    Y[q] = 0.0;
  }
}

// A^{-1} of the factored observation matrix into c->ainv (n x n; row r is
// A^{-1} e_r, and A^{-1} is symmetric), by the blocked substitutions applied
// to the rows of the identity.
cesim_status inverse_device(cesim_ctx c, hipStream_t s) {
  const int n = c->nobs;
  const size_t nn = (size_t)n * n;
  CESIM_TRY(c->ainv.reserve(sizeof(double) * nn));
  CESIM_TRY(c->ainv_tmp.reserve(sizeof(double) * nn));
  k_identity<<<(unsigned)((nn + 255) / 256), 256, 0, s>>>(c->ainv.as<double>(),
                                                          c->ainv_tmp.as<double>(), n);
  CESIM_HIP(hipGetLastError());
  CESIM_TRY(chol_solve_device(c, c->ainv.as<double>(), n, s, c->ainv_tmp.as<double>(), ST_SOLVE,
                              true));
  c->ainv_valid = true;
  return CESIM_OK;
}

// Y[r][.] = A^{-1} X[r][.] for r < R as one GEMM with c->ainv.
cesim_status apply_inverse_device(cesim_ctx c, const double* X, int R, double* Y, hipStream_t s) {
  const int n = c->nobs;
  const int tr = c->timer.begin(ST_SOLVE, s);
  GemmArgs g;
  g.M = R; g.N = n; g.K = n; g.alpha = 1.0; g.beta = 0.0;
  g.A = X; g.sai = n; g.sak = 1;
  g.B = c->ainv.as<double>(); g.sbk = n; g.sbj = 1;
  g.C = Y; g.sci = n; g.scj = 1;
  CESIM_TRY(gemm_f64(g, false, s));
  c->timer.end(tr, s);
  return CESIM_OK;
}

// ------------------------------------------- one right-hand side (GEMV form)
// The same blocked substitutions for a single vector, with dot products in
// place of GEMM tiles (a 64 x 64 tile would carry one useful row): the
// forward steps take one wave per output row (the row's entries are
// contiguous), the backward steps one lane per output column and four
// waves splitting the block's rows, reduced through LDS.

__device__ __forceinline__ double wave_sum(double a) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o);
  return a;
}

// y[i] = sum_t M[i][t] v[t] (t < nt; M rows ld apart), rows i < rows; with
// sub, y[i] = u[i] - that sum instead (u may be y).
__global__ void __launch_bounds__(256)
k_gemv_rows(const double* __restrict__ M, size_t ld, const double* __restrict__ v, int nt,
            double* y, int rows, bool sub, const double* u) {
  chain_priority();
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6), l = threadIdx.x & 63;
  if (i >= rows) return;                  // whole waves
  const double* row = M + (size_t)i * ld;
  double a = 0.0;
  for (int t = l; t < nt; t += 64) a = fma(row[t], v[t], a);
  a = wave_sum(a);
  if (l == 0) y[i] = sub ? u[i] - a : a;
}

// y[i] = sum_t M[t][i] v[t] (t < nt; M rows ld apart), columns i < cols;
// with sub, y[i] -= that sum instead.  64 columns per workgroup.
__global__ void __launch_bounds__(256)
k_gemv_cols(const double* __restrict__ M, size_t ld, const double* __restrict__ v, int nt,
            double* __restrict__ y, int cols, bool sub) {
  chain_priority();
  __shared__ double part[4][64];
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int i = blockIdx.x * 64 + l;
  double a = 0.0;
  if (i < cols) {
    // eight loads in flight per lane, the sum in row order
    int t = w;
    for (; t + 28 < nt; t += 32) {
      double m[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) m[u] = M[(size_t)(t + 4 * u) * ld + i];
#pragma unroll
      for (int u = 0; u < 8; ++u) a = fma(m[u], v[t + 4 * u], a);
    }
    for (; t < nt; t += 4) a = fma(M[(size_t)t * ld + i], v[t], a);
  }
  part[w][l] = a;
  __syncthreads();
  if (w == 0 && i < cols) {
    const double r = (part[0][l] + part[1][l]) + (part[2][l] + part[3][l]);
    y[i] = sub ? y[i] - r : r;
  }
}

// x = A^{-1} b for one vector (b is not written) with the factor in
// c->amat and the 256-block inverses in c->winv; y: n doubles of scratch.
// Same steps as chol_solve_device with R = 1; the first forward step reads
// b, so that no copy of b precedes the chain.
cesim_status chol_solve_vec_device(cesim_ctx c, const double* b, double* x, hipStream_t s,
                                   double* y, int stage) {
  const int n = c->nobs, nbig = (n + kSB - 1) / kSB;
  const double* L = c->amat.as<double>();
  const double* W = c->winv.as<double>();
  const int tr = c->timer.begin(stage, s);
  for (int kb = 0; kb < nbig; ++kb) {             // L y = b, x holding b's updated tail
    const int K0 = kb * kSB, nb = std::min(kSB, n - K0), rest = n - K0 - nb;
    const double* src = kb == 0 ? b : x;
    k_gemv_rows<<<(nb + 3) / 4, 256, 0, s>>>(W + (size_t)kb * kSB * kSB, kSB, src + K0, nb,
                                             y + K0, nb, false, nullptr);
    CESIM_HIP(hipGetLastError());
    if (rest > 0) {
      k_gemv_rows<<<(rest + 3) / 4, 256, 0, s>>>(L + (size_t)(K0 + nb) * n + K0, n, y + K0, nb,
                                                 x + K0 + nb, rest, true, src + K0 + nb);
      CESIM_HIP(hipGetLastError());
    }
  }
  for (int kb = nbig - 1; kb >= 0; --kb) {        // L^T x = y
    const int K0 = kb * kSB, nb = std::min(kSB, n - K0);
    k_gemv_cols<<<(nb + 63) / 64, 256, 0, s>>>(W + (size_t)kb * kSB * kSB, kSB, y + K0, nb, x + K0,
                                               nb, false);
    CESIM_HIP(hipGetLastError());
    if (K0 > 0) {
      k_gemv_cols<<<(K0 + 63) / 64, 256, 0, s>>>(L + (size_t)K0 * n, n, x + K0, nb, y, K0, true);
      CESIM_HIP(hipGetLastError());
    }
  }
  c->timer.end(tr, s);
  return CESIM_OK;
}

// ------------------------------------------------ grouped systems (batches)

void GroupedSeq::add_diag(const std::vector<DiagDesc>& v) {
  if (v.empty()) return;
  launches.push_back({0, (int)diag.size(), (int)v.size(), (int)v.size(), 0});
  diag.insert(diag.end(), v.begin(), v.end());
}

void GroupedSeq::add_gemm(const std::vector<GemmArgs>& v, bool lower) {
  Launch l{lower ? 2 : 1, (int)gemm.size(), 0, 0, (int)pfx.size()};
  int tiles = 0;
  for (const GemmArgs& g : v) {
    if (g.M <= 0 || g.N <= 0 || g.K <= 0) continue;
    pfx.push_back(tiles);
    tiles += ((g.M + 63) / 64) * ((g.N + 63) / 64);
    gemm.push_back(g);
    ++l.count;
  }
  if (l.count == 0) return;
  pfx.push_back(tiles);
  l.blocks = tiles;
  launches.push_back(l);
}

void GroupedSeq::clear() {
  diag.clear();
  gemm.clear();
  pfx.clear();
  launches.clear();
}

cesim_status PinnedStage::acquire(size_t n) {
  if (pending) {
    CESIM_HIP(hipEventSynchronize(done));
    pending = false;
  }
  if (!done) CESIM_HIP(hipEventCreateWithFlags(&done, hipEventDisableTiming));
  if (n <= bytes) return CESIM_OK;
  if (p) CESIM_HIP(hipHostFree(p));
  p = nullptr;
  bytes = 0;
  if (hipHostMalloc(&p, n, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    p = nullptr;
    return CESIM_ERR_OUT_OF_MEMORY;
  }
  bytes = n;
  return CESIM_OK;
}

cesim_status PinnedStage::mark(hipStream_t s) {
  CESIM_HIP(hipEventRecord(done, s));
  pending = true;
  return CESIM_OK;
}

void PinnedStage::release() {
  if (pending) (void)hipEventSynchronize(done);
  if (p) (void)hipHostFree(p);
  if (done) (void)hipEventDestroy(done);
  p = nullptr;
  bytes = 0;
  done = nullptr;
  pending = false;
}

// One contiguous table (diag | GEMMs | prefix), each part 256-byte aligned.
cesim_status GroupedSeq::upload_async(hipStream_t s, PinnedStage& st) {
  const size_t bd = sizeof(DiagDesc) * diag.size(), bg = sizeof(GemmArgs) * gemm.size();
  const size_t bp = sizeof(int) * pfx.size();
  const size_t og = (bd + 255) / 256 * 256, op = og + (bg + 255) / 256 * 256;
  const size_t total = op + bp;
  CESIM_TRY(dev.reserve(total + 256));
  CESIM_TRY(st.acquire(total));
  unsigned char* h = static_cast<unsigned char*>(st.p);
  if (bd) std::memcpy(h, diag.data(), bd);
  if (bg) std::memcpy(h + og, gemm.data(), bg);
  if (bp) std::memcpy(h + op, pfx.data(), bp);
  CESIM_HIP(hipMemcpyAsync(dev.p, h, total, hipMemcpyHostToDevice, s));
  CESIM_TRY(st.mark(s));
  unsigned char* base = dev.as<unsigned char>();
  d_diag = reinterpret_cast<DiagDesc*>(base);
  d_gemm = reinterpret_cast<GemmArgs*>(base + og);
  d_pfx = reinterpret_cast<int*>(base + op);
  return CESIM_OK;
}

cesim_status GroupedSeq::upload(hipStream_t s) {
  const size_t bd = sizeof(DiagDesc) * diag.size(), bg = sizeof(GemmArgs) * gemm.size();
  const size_t bp = sizeof(int) * pfx.size();
  const size_t og = (bd + 255) / 256 * 256, op = og + (bg + 255) / 256 * 256;
  CESIM_TRY(dev.reserve(op + bp + 256));
  unsigned char* base = dev.as<unsigned char>();
  if (bd) CESIM_HIP(hipMemcpyAsync(base, diag.data(), bd, hipMemcpyHostToDevice, s));
  if (bg) CESIM_HIP(hipMemcpyAsync(base + og, gemm.data(), bg, hipMemcpyHostToDevice, s));
  if (bp) CESIM_HIP(hipMemcpyAsync(base + op, pfx.data(), bp, hipMemcpyHostToDevice, s));
  CESIM_HIP(hipStreamSynchronize(s));
  d_diag = reinterpret_cast<DiagDesc*>(base);
  d_gemm = reinterpret_cast<GemmArgs*>(base + og);
  d_pfx = reinterpret_cast<int*>(base + op);
  return CESIM_OK;
}

cesim_status GroupedSeq::launch(hipStream_t s) const {
  for (const Launch& l : launches) {
    if (l.kind == 0)
      k_potrf_diag_grp<<<l.blocks, 256, 0, s>>>(d_diag + l.first);
    else if (l.kind == 1)
      k_gemm_f64_grp<false><<<l.blocks, 256, 0, s>>>(d_gemm + l.first, d_pfx + l.pfx, l.count);
    else
      k_gemm_f64_grp<true><<<l.blocks, 256, 0, s>>>(d_gemm + l.first, d_pfx + l.pfx, l.count);
    CESIM_HIP(hipGetLastError());
  }
  return CESIM_OK;
}

// Factor A_e = K22_e + tau_e^2 I of every context at once: step kb runs the
// diagonal block kb of every system that has one, then its panel and
// trailing update, each as one grouped launch.  The arithmetic per system
// is that of chol_factor_device.  Synchronises; not_pd[e] = 1 marks a
// non-positive pivot.
cesim_status chol_factor_batch(const std::vector<cesim_ctx>& cs, const std::vector<double>& tau2,
                               hipStream_t s, std::vector<int>& not_pd) {
  const int ne = (int)cs.size();
  not_pd.assign(ne, 0);
  int maxnb = 0;
  for (int e = 0; e < ne; ++e) {
    cesim_ctx c = cs[e];
    const int n = c->nobs, nblk = (n + kNB - 1) / kNB;
    maxnb = std::max(maxnb, nblk);
    c->yhat_valid = false;
    c->ainv_valid = false;
    CESIM_TRY(c->amat.reserve(sizeof(double) * (size_t)n * n));
    CESIM_TRY(c->dinv.reserve(sizeof(double) * (size_t)nblk * kNB * kNB));
    CESIM_HIP(hipMemsetAsync(c->chol_info.p, 0, sizeof(int) * 4, s));
    k_assemble_a<<<dim3((n + 255) / 256, n), 256, 0, s>>>(c->obs_xy.as<double>(), n, c->covd,
                                                           tau2[e], nullptr, c->amat.as<double>());
    CESIM_HIP(hipGetLastError());
  }
  GroupedSeq seq;
  for (int kb = 0; kb < maxnb; ++kb) {
    std::vector<DiagDesc> dd;
    std::vector<GemmArgs> panel, syrk;
    for (int e = 0; e < ne; ++e) {
      cesim_ctx c = cs[e];
      const int n = c->nobs, k0 = kb * kNB;
      if (k0 >= n) continue;
      const int nbk = std::min(kNB, n - k0), rest = n - k0 - nbk;
      double* A = c->amat.as<double>();
      double* D = c->dinv.as<double>() + (size_t)kb * kNB * kNB;
      dd.push_back({A, n, k0, nbk, D, c->chol_info.as<int>()});
      if (rest <= 0) continue;
      GemmArgs g;
      g.M = rest; g.N = nbk; g.K = nbk; g.alpha = 1.0; g.beta = 0.0;
      g.A = A + (size_t)(k0 + nbk) * n + k0; g.sai = n; g.sak = 1;
      g.B = D; g.sbk = 1; g.sbj = kNB;
      g.C = A + (size_t)(k0 + nbk) * n + k0; g.sci = n; g.scj = 1;
      panel.push_back(g);
      g.M = rest; g.N = rest; g.K = nbk; g.alpha = -1.0; g.beta = 1.0;
      g.A = A + (size_t)(k0 + nbk) * n + k0; g.sai = n; g.sak = 1;
      g.B = A + (size_t)(k0 + nbk) * n + k0; g.sbk = 1; g.sbj = n;
      g.C = A + (size_t)(k0 + nbk) * n + (k0 + nbk); g.sci = n; g.scj = 1;
      syrk.push_back(g);
    }
    seq.add_diag(dd);
    seq.add_gemm(panel, false);
    seq.add_gemm(syrk, true);
  }
  CESIM_TRY(seq.upload(s));
  CESIM_TRY(seq.launch(s));
  std::vector<int> flags(4 * ne);
  for (int e = 0; e < ne; ++e)
    CESIM_HIP(hipMemcpyAsync(&flags[4 * e], cs[e]->chol_info.p, sizeof(int) * 4,
                             hipMemcpyDeviceToHost, s));
  CESIM_HIP(hipStreamSynchronize(s));
  std::vector<cesim_ctx> good;
  for (int e = 0; e < ne; ++e) {
    not_pd[e] = (flags[4 * e] & 2) ? 1 : 0;
    cs[e]->chol_valid = !not_pd[e];
    cs[e]->chol_nugget = tau2[e];
    if (!not_pd[e]) good.push_back(cs[e]);
  }
  seq.dev.release();
  return build_winv(good, s);
}

// Record X_e <- A_e^{-1} X_e ([R_e][n_e], FP64) for every context with the
// factors held in the contexts: forward steps aligned at the first block,
// backward steps at each system's last block; each step's diagonal
// applications of all systems form one grouped launch, their updates the
// next.  Same GEMMs per system as chol_solve_device.
cesim_status chol_solve_batch_plan(const std::vector<cesim_ctx>& cs,
                                   const std::vector<double*>& X, const std::vector<int>& R,
                                   GroupedSeq& seq) {
  const int ne = (int)cs.size();
  std::vector<std::vector<std::vector<GemmArgs>>> fwd(ne), bwd(ne);
  int maxnb = 0;
  for (int e = 0; e < ne; ++e) {
    solve_step_lists(cs[e], X[e], cs[e]->solve_tmp.as<double>(), R[e], fwd[e], bwd[e]);
    maxnb = std::max(maxnb, (int)fwd[e].size());
  }
  for (int pass = 0; pass < 2; ++pass)
    for (int st = 0; st < maxnb; ++st)
      for (int part = 0; part < 2; ++part) {
        std::vector<GemmArgs> g;
        for (int e = 0; e < ne; ++e) {
          const auto& lst = pass == 0 ? fwd[e] : bwd[e];
          if (st < (int)lst.size() && part < (int)lst[st].size()) g.push_back(lst[st][part]);
        }
        seq.add_gemm(g, false);
      }
  return CESIM_OK;
}

}  // namespace cesim
