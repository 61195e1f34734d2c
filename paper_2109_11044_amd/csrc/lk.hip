// lk.hip -- local Kriging of the off-grid observations (Section 2.1 items
// (b)-(c); Section 3.1; Section 3.6).
//
// Setup kernel: every workgroup assembles the window covariance K11 (k x k,
// identical for all windows of a stationary field, Section 3.6) in LDS and
// factors it by Cholesky in FP64; each thread then takes one observation,
// finds its window, evaluates k_i = [C(g_alpha - s_i)], solves
// K11 w_i = k_i with the shared factor and forms
// gamma_i = C(0) - k_i^T K11^{-1} k_i = C(0) - |L^{-1} k_i|^2 (>= 0).
//
// Synthetic-data kernel (step 3): for each (realization, observation)
//   z*_{r,i} = w_i . y_r[window_i] + phi_i xi_{r,i},  phi_i = sqrt(tau^2 + gamma_i),
// with xi from Philox stream 1, and stores the right-hand side z_i - z*_{r,i}
// of the grid Kriging in FP64.
#include <hip/hip_runtime.h>

#include "internal.hpp"

namespace cesim {

template <int NPP>
__global__ void __launch_bounds__(128)
k_lk_setup(const double* __restrict__ obs, int n, GridDev g, CovDev cov, int2* __restrict__ corners,
           double* __restrict__ W, double* __restrict__ gam, int* __restrict__ info) {
  constexpr int W2 = 2 * NPP;
  constexpr int K = W2 * W2;
  __shared__ double L[K][K + 1];
  __shared__ double V[K][129];          // per-thread vectors, one column each
  // assemble K11 from index lags
  for (int e = threadIdx.x; e < K * K; e += 128) {
    const int a = e / K, b = e % K;
    const int pa = a % W2, qa = a / W2, pb = b % W2, qb = b / W2;
    L[a][b] = cov_eval(cov, (double)(pa - pb) * g.dx, (double)(qa - qb) * g.dy);
  }
  __syncthreads();
  // right-looking Cholesky, lower triangle
  for (int j = 0; j < K; ++j) {
    if (threadIdx.x == 0) {
      const double d = L[j][j];
      if (!(d > 0.0) && blockIdx.x == 0) atomicOr(info, 1);
      L[j][j] = sqrt(d);
    }
    __syncthreads();
    for (int i = j + 1 + threadIdx.x; i < K; i += 128) L[i][j] /= L[j][j];
    __syncthreads();
    const int rem = K - j - 1;
    for (int e = threadIdx.x; e < rem * rem; e += 128) {
      const int i = j + 1 + e / rem, l = j + 1 + e % rem;
      if (l <= i) L[i][l] -= L[i][j] * L[l][j];
    }
    __syncthreads();
  }
  const int i = blockIdx.x * 128 + threadIdx.x;
  if (i >= n) return;
  const double sx = obs[2 * i], sy = obs[2 * i + 1];
  int a = (int)floor((sx - g.x0) / g.dx) - NPP + 1;
  int b = (int)floor((sy - g.y0) / g.dy) - NPP + 1;
  a = min(max(a, 0), g.m1 - W2);
  b = min(max(b, 0), g.m2 - W2);
  // this thread's vector lives in LDS column threadIdx.x (conflict-free)
  double* v = &V[0][threadIdx.x];
  constexpr int LD = 129;
  for (int al = 0; al < K; ++al) {
    const int p = al % W2, q = al / W2;
    // node coordinate written out without contraction, as x0 + i dx
    const double gx = __dadd_rn(g.x0, __dmul_rn((double)(a + p), g.dx));
    const double gy = __dadd_rn(g.y0, __dmul_rn((double)(b + q), g.dy));
    v[al * LD] = cov_eval(cov, gx - sx, gy - sy);
  }
  // forward substitution: v <- L^{-1} k; gamma = C(0) - |L^{-1} k|^2
  double ss = 0.0;
  for (int al = 0; al < K; ++al) {
    double t = v[al * LD];
    for (int be = 0; be < al; ++be) t -= L[al][be] * v[be * LD];
    t /= L[al][al];
    v[al * LD] = t;
    ss += t * t;
  }
  // back substitution: v <- L^{-T} v = K11^{-1} k
  for (int al = K - 1; al >= 0; --al) {
    double t = v[al * LD];
    for (int be = al + 1; be < K; ++be) t -= L[be][al] * v[be * LD];
    v[al * LD] = t / L[al][al];
  }
  for (int al = 0; al < K; ++al) W[(size_t)i * K + al] = v[al * LD];
  gam[i] = fmax(0.0, cov.sigma2 - ss);
  corners[i] = make_int2(a, b);
}

// Local Kriging on the mean noise and its derivatives, for the gradient of
// a linear ensemble statistic (Section 2.1 (b)-(c) differentiated).  One
// thread per observation i, 64 per workgroup sharing the factor L of K11
// (dynamic LDS: L, then two columns of K doubles per thread):
//   w_i = K11^{-1} k_i,  gamma_i = C(0) - |L^{-1} k_i|^2 (>= 0),
//   dw_i = K11^{-1} (dk_i - dK11 w_i),  dgamma_i = -2 dk_i . w_i + w_i . dK11 w_i
// (dK11, dk_i: theta-derivatives; dK11 is evaluated where it is used), and
// with phi_i = sqrt(tau^2 + gamma_i), xi = xib[i] and the window values of
// yb and dyb:
//   out[4i]     = w_i . yb[N_i] + phi_i xi                       (zbar*_i)
//   out[4i + 1] = dw_i . yb[N_i] + w_i . dyb[N_i] + xi dgamma_i / (2 phi_i)
//   out[4i + 2] = w_i . yb[N_i] / (2 sigma^2) + xi gamma_i / (2 sigma^2 phi_i)
//   out[4i + 3] = xi / (2 phi_i)
// (the theta-, sigma^2- and tau^2-derivatives of zbar*_i).
template <int NPP>
__global__ void __launch_bounds__(64)
k_lk_grad(const double* __restrict__ obs, int n, GridDev g, CovDev cov, double tau2,
          const double* __restrict__ yb, const double* __restrict__ dyb,
          const double* __restrict__ xib, double* __restrict__ out) {
  constexpr int W2 = 2 * NPP;
  constexpr int K = W2 * W2;
  constexpr int LD = 65;
  extern __shared__ double sm[];
  double (*L)[K + 1] = reinterpret_cast<double (*)[K + 1]>(sm);
  double* V = sm + K * (K + 1);                 // [K][LD]: k_i, then w_i
  double* U = V + K * LD;                       // [K][LD]: dk_i, then dw_i
  for (int e = threadIdx.x; e < K * K; e += 64) {
    const int a = e / K, b = e % K;
    L[a][b] = cov_eval(cov, (double)(a % W2 - b % W2) * g.dx, (double)(a / W2 - b / W2) * g.dy);
  }
  __syncthreads();
  for (int j = 0; j < K; ++j) {
    if (threadIdx.x == 0) L[j][j] = sqrt(L[j][j]);   // positive: checked at set-up
    __syncthreads();
    for (int i = j + 1 + threadIdx.x; i < K; i += 64) L[i][j] /= L[j][j];
    __syncthreads();
    const int rem = K - j - 1;
    for (int e = threadIdx.x; e < rem * rem; e += 64) {
      const int i = j + 1 + e / rem, l = j + 1 + e % rem;
      if (l <= i) L[i][l] -= L[i][j] * L[l][j];
    }
    __syncthreads();
  }
  const int i = blockIdx.x * 64 + threadIdx.x;
  if (i >= n) return;
  const double sx = obs[2 * i], sy = obs[2 * i + 1];
  int a = (int)floor((sx - g.x0) / g.dx) - NPP + 1;
  int b = (int)floor((sy - g.y0) / g.dy) - NPP + 1;
  a = min(max(a, 0), g.m1 - W2);
  b = min(max(b, 0), g.m2 - W2);
  double* v = V + threadIdx.x;
  double* u = U + threadIdx.x;
  for (int al = 0; al < K; ++al) {
    const double gx = __dadd_rn(g.x0, __dmul_rn((double)(a + al % W2), g.dx));
    const double gy = __dadd_rn(g.y0, __dmul_rn((double)(b + al / W2), g.dy));
    v[al * LD] = cov_eval(cov, gx - sx, gy - sy);
    u[al * LD] = dcov_eval(cov, gx - sx, gy - sy);
  }
  auto solve = [&](double* x, double* ss) {     // x <- K11^{-1} x; ss = |L^{-1} x|^2
    double acc = 0.0;
    for (int al = 0; al < K; ++al) {
      double t = x[al * LD];
      for (int be = 0; be < al; ++be) t -= L[al][be] * x[be * LD];
      t /= L[al][al];
      x[al * LD] = t;
      acc += t * t;
    }
    for (int al = K - 1; al >= 0; --al) {
      double t = x[al * LD];
      for (int be = al + 1; be < K; ++be) t -= L[be][al] * x[be * LD];
      x[al * LD] = t / L[al][al];
    }
    if (ss) *ss = acc;
  };
  double ss;
  solve(v, &ss);                                // v = w_i
  double dkw = 0.0, wdkw = 0.0;
  for (int al = 0; al < K; ++al) {
    double r = 0.0;                             // (dK11 w)_al
    for (int be = 0; be < K; ++be)
      r += dcov_eval(cov, (double)(al % W2 - be % W2) * g.dx, (double)(al / W2 - be / W2) * g.dy) *
           v[be * LD];
    dkw += u[al * LD] * v[al * LD];
    wdkw += v[al * LD] * r;
    u[al * LD] -= r;
  }
  solve(u, nullptr);                            // u = dw_i
  const double gam = fmax(0.0, cov.sigma2 - ss);
  const double dgam = gam > 0.0 ? wdkw - 2.0 * dkw : 0.0;
  double wy = 0.0, wdy = 0.0, dwy = 0.0;
  for (int al = 0; al < K; ++al) {
    const size_t node = (size_t)(b + al / W2) * g.m1 + (a + al % W2);
    wy += v[al * LD] * yb[node];
    wdy += v[al * LD] * dyb[node];
    dwy += u[al * LD] * yb[node];
  }
  const double phi = sqrt(tau2 + gam), xi = xib[i], s2 = cov.sigma2;
  out[4 * (size_t)i] = wy + phi * xi;
  out[4 * (size_t)i + 1] = dwy + wdy + xi * dgam / (2.0 * phi);
  out[4 * (size_t)i + 2] = wy / (2.0 * s2) + xi * gam / (2.0 * s2 * phi);
  out[4 * (size_t)i + 3] = xi / (2.0 * phi);
}

cesim_status lk_grad_device(cesim_ctx c, double tau2, const double* yb, const double* dyb,
                            const double* xib, double* out) {
  hipStream_t s = c->stream;
  const int n = c->nobs, K = c->k;
  const size_t lds = sizeof(double) * ((size_t)K * (K + 1) + 2 * (size_t)K * 65);
  const dim3 grid((n + 63) / 64);
  auto go = [&](auto kern) -> cesim_status {
    if (lds > 64 * 1024)
      CESIM_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    kern<<<grid, 64, lds, s>>>(c->obs_xy.as<double>(), n, c->gridd, c->covd, tau2, yb, dyb, xib,
                               out);
    CESIM_HIP(hipGetLastError());
    return CESIM_OK;
  };
  switch (c->npp) {
    case 1: return go(k_lk_grad<1>);
    case 2: return go(k_lk_grad<2>);
    case 3: return go(k_lk_grad<3>);
    default: return go(k_lk_grad<4>);
  }
}

__global__ void k_phi(const double* __restrict__ gam, int n, double tau2, double* __restrict__ phi) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) phi[i] = sqrt(tau2 + gam[i]);
}

// rhs[r][i] = z_i - (w_i . y_r[window_i] + phi_i xi_{r,i})   (z_i = 0 when z is null)
template <typename F>
__global__ void __launch_bounds__(256)
k_synth_rhs(const F* __restrict__ fields, int m1, int m2, const int2* __restrict__ corners,
            const double* __restrict__ W, const double* __restrict__ phi,
            const double* __restrict__ z, int n, int K, int w2, NoiseKey key,
            const int* __restrict__ order, double* __restrict__ rhs) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  const int r = blockIdx.y;
  if (t >= n) return;
  // observations in spatial order: neighbouring lanes gather from
  // neighbouring windows and share cache lines (results are per observation)
  const int i = order[t];
  const int2 ab = corners[i];
  const F* y = fields + (size_t)r * m1 * m2 + (size_t)ab.y * m1 + ab.x;
  const double* w = W + (size_t)i * K;
  double acc = 0.0;
  for (int q = 0; q < w2; ++q)
    for (int p = 0; p < w2; ++p) acc += w[q * w2 + p] * (double)y[(size_t)q * m1 + p];
  // xi_{r,i}: block i/4, word i%4 of Philox stream 1
  const u32x4 wd = philox4x32_10({(uint32_t)(i >> 2), (uint32_t)(key.base() + r), key.event, 1u},
                                 key.k0, key.k1);
  const int word = i & 3;
  double z0, z1;
  if (word < 2) box_muller_f64(wd.x, wd.y, z0, z1);
  else box_muller_f64(wd.z, wd.w, z0, z1);
  const double xi = (word & 1) ? z1 : z0;
  rhs[(size_t)r * n + i] = (z ? z[i] : 0.0) - (acc + phi[i] * xi);
}

cesim_status lk_setup_device(cesim_ctx c) {
  hipStream_t s = c->stream;
  const int n = c->nobs;
  CESIM_HIP(hipMemsetAsync(c->info_dev.p, 0, sizeof(int) * 4, s));
  dim3 grid((n + 127) / 128);
  int* info = c->info_dev.as<int>();
  auto* obs = c->obs_xy.as<double>();
  auto* cor = c->corners.as<int2>();
  auto* W = c->weights.as<double>();
  auto* gm = c->gamma.as<double>();
  const int tr = c->timer.begin(ST_LK_SETUP, s);
  switch (c->npp) {
    case 1: k_lk_setup<1><<<grid, 128, 0, s>>>(obs, n, c->gridd, c->covd, cor, W, gm, info); break;
    case 2: k_lk_setup<2><<<grid, 128, 0, s>>>(obs, n, c->gridd, c->covd, cor, W, gm, info); break;
    case 3: k_lk_setup<3><<<grid, 128, 0, s>>>(obs, n, c->gridd, c->covd, cor, W, gm, info); break;
    case 4: k_lk_setup<4><<<grid, 128, 0, s>>>(obs, n, c->gridd, c->covd, cor, W, gm, info); break;
    default: return CESIM_ERR_INVALID_ARG;
  }
  CESIM_HIP(hipGetLastError());
  c->timer.end(tr, s);
  return CESIM_OK;
}

cesim_status lk_phi_device(cesim_ctx c, double tau2) {
  const int tr = c->timer.begin(ST_SYNTH_RHS, c->stream);
  k_phi<<<(c->nobs + 255) / 256, 256, 0, c->stream>>>(c->gamma.as<double>(), c->nobs, tau2,
                                                      c->phi.as<double>());
  CESIM_HIP(hipGetLastError());
  c->timer.end(tr, c->stream);
  return CESIM_OK;
}

cesim_status lk_synth_rhs_device(cesim_ctx c, const void* fields, double* rhs, bool with_z) {
  const double* z = with_z ? c->zdev.as<double>() : nullptr;
  const int n = c->nobs;
  dim3 grid((n + 255) / 256, c->nreal);
  const NoiseKey key{(uint32_t)(c->seed & 0xffffffffu), (uint32_t)(c->seed >> 32), c->first_real,
                     c->event_id, c->roff};
  const int w2 = 2 * c->npp;
  const int tr = c->timer.begin(ST_SYNTH_RHS, c->stream);
  if (c->prec == CESIM_PREC_FP64)
    k_synth_rhs<double><<<grid, 256, 0, c->stream>>>(
        static_cast<const double*>(fields), c->grid.m1, c->grid.m2, c->corners.as<int2>(),
        c->weights.as<double>(), c->phi.as<double>(), z, n, c->k, w2, key,
        c->obs_order.as<int>(), rhs);
  else
    k_synth_rhs<float><<<grid, 256, 0, c->stream>>>(
        static_cast<const float*>(fields), c->grid.m1, c->grid.m2, c->corners.as<int2>(),
        c->weights.as<double>(), c->phi.as<double>(), z, n, c->k, w2, key,
        c->obs_order.as<int>(), rhs);
  CESIM_HIP(hipGetLastError());
  c->timer.end(tr, c->stream);
  return CESIM_OK;
}

}  // namespace cesim
