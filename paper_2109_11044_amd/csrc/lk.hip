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
// (the theta-, sigma^2- and tau^2-derivatives of zbar*_i), for R sets of
// fields and noises at once (set r: yb + r M, dyb + r M, xib + r n,
// out + 4 r n; the weights and their derivatives are computed once).
template <int NPP>
__global__ void __launch_bounds__(64)
k_lk_grad(const double* __restrict__ obs, int n, GridDev g, CovDev cov, double tau2,
          const double* __restrict__ yb, const double* __restrict__ dyb,
          const double* __restrict__ xib, double* __restrict__ out, int R) {
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
  const double phi = sqrt(tau2 + gam), s2 = cov.sigma2;
  // phi = 0 only with tau^2 = 0 and gamma_i = 0 (the host refuses that
  // case for the nugget derivative); gamma and its derivative vanish there,
  // so the noise terms of the range and sigma^2 derivatives are 0
  const double hphi = phi > 0.0 ? 0.5 / phi : 0.0;
  const size_t M = (size_t)g.m1 * g.m2;
  for (int r = 0; r < R; ++r) {
    const double* y = yb + r * M;
    const double* dy = dyb + r * M;
    double wy = 0.0, wdy = 0.0, dwy = 0.0;
    for (int al = 0; al < K; ++al) {
      const size_t node = (size_t)(b + al / W2) * g.m1 + (a + al % W2);
      wy += v[al * LD] * y[node];
      wdy += v[al * LD] * dy[node];
      dwy += u[al * LD] * y[node];
    }
    const double xi = xib[(size_t)r * n + i];
    double* o = out + 4 * ((size_t)r * n + i);
    o[0] = wy + phi * xi;
    o[1] = dwy + wdy + xi * dgam * hphi;
    o[2] = wy / (2.0 * s2) + xi * gam * hphi / s2;
    o[3] = xi * hphi;
  }
}

cesim_status lk_grad_device(cesim_ctx c, double tau2, const double* yb, const double* dyb,
                            const double* xib, double* out, int R) {
  hipStream_t s = c->stream;
  const int n = c->nobs, K = c->k;
  const size_t lds = sizeof(double) * ((size_t)K * (K + 1) + 2 * (size_t)K * 65);
  const dim3 grid((n + 63) / 64);
  auto go = [&](auto kern) -> cesim_status {
    if (lds > 64 * 1024)
      CESIM_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    kern<<<grid, 64, lds, s>>>(c->obs_xy.as<double>(), n, c->gridd, c->covd, tau2, yb, dyb, xib,
                               out, R);
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

// xi_{r,i}: block i/4, word i%4 of Philox stream 1.
__device__ inline double obs_normal(const NoiseKey& key, int r, int i) {
  const u32x4 wd = philox4x32_10({(uint32_t)(i >> 2), (uint32_t)(key.base() + r), key.event, 1u},
                                 key.k0, key.k1);
  const int word = i & 3;
  double z0, z1;
  if (word < 2) box_muller_f64(wd.x, wd.y, z0, z1);
  else box_muller_f64(wd.z, wd.w, z0, z1);
  return (word & 1) ? z1 : z0;
}

// Boxes of several observations (joint sampling): for observation i,
// box[i] = {descriptor index, row within the box} or {-1, 0}; descriptor d
// = {first member in `members`, size, offset of the packed factor};
// members: observation indices of each box in ascending order.
struct JointBoxes {
  const int2* box;
  const int4* desc;
  const int* members;
  const double* fac;            // packed lower factors, row p at p (p + 1) / 2
};

// rhs[r][i] = z_i - (w_i . y_r[window_i] + e_{r,i})   (z_i = 0 when z is null)
// e_{r,i} = phi_i xi_{r,i}, or with JOINT for a member of a box of several
// observations, row p of L_G xi_{r,G}.  W2: the window width 2 n_p, fixed
// at compile time so that all W2^2 gathers of a thread are in flight at once.
constexpr int kMaxBox = kMaxJointBox;
template <typename F, bool JOINT, int W2>
__global__ void __launch_bounds__(256)
k_synth_rhs(const F* __restrict__ fields, int m1, int m2, const int2* __restrict__ corners,
            const double* __restrict__ W, const double* __restrict__ phi,
            const double* __restrict__ z, int n, NoiseKey key,
            const int* __restrict__ order, double* __restrict__ rhs, JointBoxes jb) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  const int r = blockIdx.y;
  if (t >= n) return;
  // observations in spatial order: neighbouring lanes gather from
  // neighbouring windows and share cache lines (results are per observation)
  const int i = order[t];
  const int2 ab = corners[i];
  const F* y = fields + (size_t)r * m1 * m2 + (size_t)ab.y * m1 + ab.x;
  const double* w = W + (size_t)i * (W2 * W2);
  F v[W2 * W2];
#pragma unroll
  for (int q = 0; q < W2; ++q)
#pragma unroll
    for (int p = 0; p < W2; ++p) v[q * W2 + p] = y[(size_t)q * m1 + p];
  double acc = 0.0;
#pragma unroll
  for (int a = 0; a < W2 * W2; ++a) acc += w[a] * (double)v[a];
  double e;
  const int2 bx = JOINT ? jb.box[i] : make_int2(-1, 0);
  if (bx.x < 0) {
    e = phi[i] * obs_normal(key, r, i);
  } else {
    const int4 d = jb.desc[bx.x];
    const double* Lrow = jb.fac + d.z + bx.y * (bx.y + 1) / 2;
    e = 0.0;
    for (int q = 0; q <= bx.y; ++q) e += Lrow[q] * obs_normal(key, r, jb.members[d.x + q]);
  }
  rhs[(size_t)r * n + i] = (z ? z[i] : 0.0) - (acc + e);
}

// Factor of every box of several observations: one workgroup per box,
// G = size <= kMaxBox members sharing the window of the first.  Gamma_ij =
// C(s_i - s_j) - w_i . k_j (k_j: covariances between the window nodes and
// s_j), plus tau^2 on the diagonal; Cholesky, packed lower factor.  Bit 4 of
// *info marks a non-positive pivot.
template <int NPP>
__global__ void __launch_bounds__(64)
k_box_factor(const double* __restrict__ obs, GridDev g, CovDev cov, const int2* __restrict__ corners,
             const double* __restrict__ W, double tau2, JointBoxes jb, double* __restrict__ fac,
             int* __restrict__ info) {
  constexpr int W2 = 2 * NPP;
  constexpr int K = W2 * W2;
  __shared__ double kc[K][kMaxBox + 1];   // column j: k_j
  __shared__ double Gm[kMaxBox][kMaxBox + 1];
  const int4 d = jb.desc[blockIdx.x];
  const int G = d.y, t = threadIdx.x;
  const int i0 = jb.members[d.x];
  const int2 ab = corners[i0];
  if (t < G) {
    const int j = jb.members[d.x + t];
    const double sx = obs[2 * j], sy = obs[2 * j + 1];
    for (int al = 0; al < K; ++al) {
      const double gx = __dadd_rn(g.x0, __dmul_rn((double)(ab.x + al % W2), g.dx));
      const double gy = __dadd_rn(g.y0, __dmul_rn((double)(ab.y + al / W2), g.dy));
      kc[al][t] = cov_eval(cov, gx - sx, gy - sy);
    }
  }
  __syncthreads();
  if (t < G) {                             // row t of Gamma (lower part)
    const int it = jb.members[d.x + t];
    const double* w = W + (size_t)it * K;
    for (int jj = 0; jj <= t; ++jj) {
      const int j = jb.members[d.x + jj];
      double acc = 0.0;
      for (int al = 0; al < K; ++al) acc += w[al] * kc[al][jj];
      Gm[t][jj] = cov_eval(cov, obs[2 * it] - obs[2 * j], obs[2 * it + 1] - obs[2 * j + 1]) - acc +
                  (jj == t ? tau2 : 0.0);
    }
  }
  __syncthreads();
  for (int j = 0; j < G; ++j) {           // right-looking Cholesky, lower triangle
    if (t == 0) {
      const double dj = Gm[j][j];
      if (!(dj > 0.0)) atomicOr(info, 2);
      Gm[j][j] = sqrt(dj);
    }
    __syncthreads();
    if (t > j && t < G) Gm[t][j] /= Gm[j][j];
    __syncthreads();
    if (t > j && t < G)
      for (int l = j + 1; l <= t; ++l) Gm[t][l] -= Gm[t][j] * Gm[l][j];
    __syncthreads();
  }
  if (t < G)
    for (int q = 0; q <= t; ++q) fac[d.z + t * (t + 1) / 2 + q] = Gm[t][q];
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

static JointBoxes joint_boxes(cesim_ctx c) {
  return {c->box_of.as<int2>(), c->box_desc.as<int4>(), c->box_members.as<int>(),
          c->box_fac.as<double>()};
}

// Joint sampling is in force when it is switched on and some box holds
// several observations.
bool joint_active(cesim_ctx c) { return c->joint_boxes && c->nboxes > 0; }

cesim_status lk_synth_rhs_device(cesim_ctx c, const void* fields, double* rhs, bool with_z) {
  const double* z = with_z ? c->zdev.as<double>() : nullptr;
  const int n = c->nobs;
  dim3 grid((n + 255) / 256, c->nreal);
  const NoiseKey key{(uint32_t)(c->seed & 0xffffffffu), (uint32_t)(c->seed >> 32), c->first_real,
                     c->event_id, c->roff};
  const JointBoxes jb = joint_boxes(c);
  const int tr = c->timer.begin(ST_SYNTH_RHS, c->stream);
#define CESIM_SYNTH_W(F, J, W2)                                                                     \
  k_synth_rhs<F, J, W2><<<grid, 256, 0, c->stream>>>(                                               \
      static_cast<const F*>(fields), c->grid.m1, c->grid.m2, c->corners.as<int2>(),                \
      c->weights.as<double>(), c->phi.as<double>(), z, n, key, c->obs_order.as<int>(), rhs, jb)
#define CESIM_SYNTH(F, J)                                 \
  switch (c->npp) {                                       \
    case 1: CESIM_SYNTH_W(F, J, 2); break;                \
    case 2: CESIM_SYNTH_W(F, J, 4); break;                \
    case 3: CESIM_SYNTH_W(F, J, 6); break;                \
    default: CESIM_SYNTH_W(F, J, 8); break;               \
  }
  if (c->prec == CESIM_PREC_FP64) {
    if (joint_active(c)) { CESIM_SYNTH(double, true) }
    else { CESIM_SYNTH(double, false) }
  } else {
    if (joint_active(c)) { CESIM_SYNTH(float, true) }
    else { CESIM_SYNTH(float, false) }
  }
#undef CESIM_SYNTH
#undef CESIM_SYNTH_W
  CESIM_HIP(hipGetLastError());
  c->timer.end(tr, c->stream);
  return CESIM_OK;
}

// Factors of the boxes of several observations for nugget tau2 (joint
// sampling), on stream s; a non-positive pivot sets bit 2 of c->chol_info[0]
// (the flag of the observation factorisation, cleared by the caller).
cesim_status box_factor_device(cesim_ctx c, double tau2, hipStream_t s) {
  if (!joint_active(c)) return CESIM_OK;
  if (c->max_box > kMaxBox) return CESIM_ERR_INVALID_ARG;
  const JointBoxes jb = joint_boxes(c);
  int* info = c->chol_info.as<int>();
  const dim3 grid(c->nboxes);
#define CESIM_BOXF(NP)                                                                         \
  k_box_factor<NP><<<grid, 64, 0, s>>>(c->obs_xy.as<double>(), c->gridd, c->covd,             \
                                       c->corners.as<int2>(), c->weights.as<double>(), tau2, jb, \
                                       c->box_fac.as<double>(), info)
  switch (c->npp) {
    case 1: CESIM_BOXF(1); break;
    case 2: CESIM_BOXF(2); break;
    case 3: CESIM_BOXF(3); break;
    default: CESIM_BOXF(4); break;
  }
#undef CESIM_BOXF
  CESIM_HIP(hipGetLastError());
  return CESIM_OK;
}

}  // namespace cesim
