// grad.hip -- gradient of a linear ensemble statistic of the conditional
// realizations (steps 1-5 of Section 2 with the local Kriging of
// Section 2.1; eq. (4)), FP64:
//   L = (1/R) sum_r sum_g w_g v_r[g]
// with respect to the range theta, the sill sigma^2, the nugget tau^2 and the
// observed values z.  Every v_r is affine in its noise (the pair noise
// zeta_{r/2} of the draw, y_r = Re(c_r FFT2(sqrt(lambda / N) zeta_{r/2})) with
// c_r = 1 or -i, and xi_r of the synthetic data), so L and its derivatives
// follow from one evaluation on the mean noises zeta_bar, xi_bar:
//   ybar  = crop(Re FFT2(sqrt(lambda / N) zeta_bar)),  zbar* = W1 ybar + phi xi_bar,
//   L     = w . ybar + u . (z - zbar*),  u = A^{-1} p,  p = K21 w,  A = K22 + tau^2 I.
// With cbar = A^{-1} (z - zbar*) and dA^{-1} = -A^{-1} dA A^{-1}:
//   dL/dz      = u
//   dL/dtau^2  = -u . cbar - u . t_tau
//   dL/dsigma^2 = w . ybar / (2 sigma^2) + p . cbar / sigma^2
//                 - (u . (z - zbar*) - tau^2 u . cbar) / sigma^2 - u . t_sigma
//   dL/dtheta  = w . dybar + dp . cbar - u . (dK22 cbar) - u . t_theta
// where t_* are the derivatives of zbar* (local-Kriging kernel k_lk_grad),
// dybar the draw with d sqrt(lambda)/dtheta, dp = dK21 w and dK22 the
// theta-derivatives of the cross- and observation covariances.
//
// The vector-Jacobian product of the fields themselves (the gradient of any
// ensemble statistic, given its derivatives vbar[r] with respect to each
// v_r) is the sum over r of this linear statistic for realization r alone
// with weights vbar[r].
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "internal.hpp"

namespace cesim {

namespace {

// zeta_bar[q] = mean over r of c_r zeta_{r/2}[q]: zeta_P = eps_{2P} + i
// eps_{2P+1} is the pair noise of torus element q (stream 0: block q / 4,
// word q % 4) and c_r = 1 (r even) or -i (r odd), so that y_r = Re(c_r W_P),
// r = first .. first + R - 1.
__global__ void k_mean_pair_noise(uint32_t k0, uint32_t k1, uint32_t event, int first, int R,
                                  size_t N, double2* __restrict__ zb) {
  const size_t blk = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (blk * 4 >= N) return;
  double ar[4] = {0.0, 0.0, 0.0, 0.0}, ai[4] = {0.0, 0.0, 0.0, 0.0};
  const int last = first + R - 1;
  for (int P = first >> 1; P <= last >> 1; ++P) {
    double za[4], zo[4];
    normals4_f64(k0, k1, (uint32_t)blk, (uint32_t)(2 * P), event, 0u, za);
    normals4_f64(k0, k1, (uint32_t)blk, (uint32_t)(2 * P + 1), event, 0u, zo);
    const bool even = 2 * P >= first, odd = 2 * P + 1 <= last;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      if (even) { ar[w] += za[w]; ai[w] += zo[w]; }
      if (odd) { ar[w] += zo[w]; ai[w] -= za[w]; }
    }
  }
#pragma unroll
  for (int w = 0; w < 4; ++w)
    if (blk * 4 + w < N) zb[blk * 4 + w] = {ar[w] / (double)R, ai[w] / (double)R};
}

// xi_bar[i] = mean over r of the stream-1 normal of observation i.
__global__ void k_mean_obs_noise(uint32_t k0, uint32_t k1, uint32_t event, int first, int R,
                                 int n, double* __restrict__ xb) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  double acc = 0.0;
  for (int r = 0; r < R; ++r) {
    double z[4];
    normals4_f64(k0, k1, (uint32_t)(i >> 2), (uint32_t)(first + r), event, 1u, z);
    acc += z[i & 3];
  }
  xb[i] = acc / (double)R;
}

// p_i = sum_g C(s_i - g) w_g and dp_i = sum_g dC(s_i - g)/dtheta w_g: one
// workgroup per observation, fixed-order reduction.
__global__ void __launch_bounds__(256)
k_cross_gemv(const double* __restrict__ obs, GridDev g, CovDev cov, const double* __restrict__ w,
             double* __restrict__ p, double* __restrict__ dp) {
  __shared__ double r0[256], r1[256];
  const int i = blockIdx.x;
  const double sx = obs[2 * i], sy = obs[2 * i + 1];
  const int M = g.m1 * g.m2;
  double a = 0.0, b = 0.0;
  for (int q = threadIdx.x; q < M; q += 256) {
    const int x = q % g.m1, y = q / g.m1;
    const double hx = __dadd_rn(g.x0, __dmul_rn((double)x, g.dx)) - sx;
    const double hy = __dadd_rn(g.y0, __dmul_rn((double)y, g.dy)) - sy;
    const double wq = w[q];
    double cv, dv;
    cov_dcov_eval(cov, hx, hy, cv, dv);
    a += cv * wq;
    b += dv * wq;
  }
  r0[threadIdx.x] = a;
  r1[threadIdx.x] = b;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) {
      r0[threadIdx.x] += r0[threadIdx.x + h];
      r1[threadIdx.x] += r1[threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    p[i] = r0[0];
    dp[i] = r1[0];
  }
}

// q_i = sum_j dC(s_i - s_j)/dtheta c_j (the theta-derivative of K22 times c).
__global__ void __launch_bounds__(256)
k_dk22_times(const double* __restrict__ obs, int n, CovDev cov, const double* __restrict__ c,
             double* __restrict__ q) {
  __shared__ double red[256];
  const int i = blockIdx.x;
  const double sx = obs[2 * i], sy = obs[2 * i + 1];
  double a = 0.0;
  for (int j = threadIdx.x; j < n; j += 256)
    a += dcov_eval(cov, sx - obs[2 * j], sy - obs[2 * j + 1]) * c[j];
  red[threadIdx.x] = a;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) q[i] = red[0];
}

// rhs rows of the solve: row 0 = p, row 1 = z - zbar* (zbar*_i = t[4 i]).
__global__ void k_grad_rhs(const double* __restrict__ p, const double* __restrict__ z,
                           const double* __restrict__ t, int n, double* __restrict__ X) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  X[i] = p[i];
  X[n + i] = z[i] - t[4 * (size_t)i];
}

constexpr int kDots = 11;
struct DotList {
  const double* a[kDots];
  const double* b[kDots];
  int sb[kDots];      // element stride of b
  int len[kDots];
};

// out[k] = sum_i a_k[i] b_k[i sb_k], one workgroup per product, fixed order.
__global__ void __launch_bounds__(256) k_dots(DotList d, double* __restrict__ out) {
  __shared__ double red[256];
  const int k = blockIdx.x;
  const double* a = d.a[k];
  const double* b = d.b[k];
  double acc = 0.0;
  for (int i = threadIdx.x; i < d.len[k]; i += 256) acc += a[i] * b[(size_t)i * d.sb[k]];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[k] = red[0];
}

// xi[r][i]: the stream-1 normal of observation i in realization first + r.
__global__ void k_obs_noise_all(uint32_t k0, uint32_t k1, uint32_t event, int first, int R, int n,
                                double* __restrict__ xi) {
  const size_t q = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (q >= (size_t)R * n) return;
  const int r = (int)(q / n), i = (int)(q % n);
  double z[4];
  normals4_f64(k0, k1, (uint32_t)(i >> 2), (uint32_t)(first + r), event, 1u, z);
  xi[q] = z[i & 3];
}

// Partial cross products over one segment of grid nodes:
//   Pp[z][r][i] = sum_{g in segment z} C(s_i - g) vbar[r][g],
//   dPp[z][r][i] = the same with dC(s_i - g)/dtheta,
// for r < R, i < n.  Workgroup (bx, by, z): stations 16 bx .. + 15,
// realizations 256 by .. + 255, nodes [z seg, (z + 1) seg) in chunks of 16.
// Per chunk the 16 x 16 covariances and derivatives (one per thread) and
// the 256 x 16 tile of vbar go to LDS; thread t accumulates station t % 16
// for realizations 16 (t / 16) .. + 15, so each covariance serves 256
// realizations.  k_cross_adj_sum adds the segments in order.
__global__ void __launch_bounds__(256)
k_cross_adj(const double* __restrict__ obs, int n, GridDev g, CovDev cov,
            const double* __restrict__ vbar, int R, int seg, double* __restrict__ Pp,
            double* __restrict__ dPp) {
  __shared__ double Cs[16][17], dCs[16][17];
  __shared__ double V[256][17];
  const int t = threadIdx.x;
  const int i0 = blockIdx.x * 16, r0 = blockIdx.y * 256, z = blockIdx.z;
  const int M = g.m1 * g.m2;
  const int gb = z * seg, ge = min(M, gb + seg);
  const int il = t & 15, rg = (t >> 4) * 16;
  double ap[16], ad[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) ap[q] = ad[q] = 0.0;
  for (int g0 = gb; g0 < ge; g0 += 16) {
    __syncthreads();
    {
      const int gl = t >> 4, sl = t & 15;
      const int gg = g0 + gl, ii = i0 + sl;
      double cv = 0.0, dv = 0.0;
      if (gg < ge && ii < n) {
        const int x = gg % g.m1, y = gg / g.m1;
        const double hx = __dadd_rn(g.x0, __dmul_rn((double)x, g.dx)) - obs[2 * ii];
        const double hy = __dadd_rn(g.y0, __dmul_rn((double)y, g.dy)) - obs[2 * ii + 1];
        cov_dcov_eval(cov, hx, hy, cv, dv);
      }
      Cs[gl][sl] = cv;
      dCs[gl][sl] = dv;
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = t + 256 * u, rl = e >> 4, gl = e & 15;
      const int rr = r0 + rl, gg = g0 + gl;
      V[rl][gl] = (rr < R && gg < ge) ? vbar[(size_t)rr * M + gg] : 0.0;
    }
    __syncthreads();
#pragma unroll 2
    for (int gl = 0; gl < 16; ++gl) {
      const double cv = Cs[gl][il], dv = dCs[gl][il];
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const double v = V[rg + q][gl];
        ap[q] = fma(v, cv, ap[q]);
        ad[q] = fma(v, dv, ad[q]);
      }
    }
  }
  const int ii = i0 + il;
  if (ii >= n) return;
  const size_t base = (size_t)z * R * n;
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int rr = r0 + rg + q;
    if (rr < R) {
      Pp[base + (size_t)rr * n + ii] = ap[q];
      dPp[base + (size_t)rr * n + ii] = ad[q];
    }
  }
}

// P[q] = sum_z Pp[z][q], dP likewise (q < R n), segments in order.
__global__ void k_cross_adj_sum(const double* __restrict__ Pp, const double* __restrict__ dPp,
                                int S, size_t Rn, double* __restrict__ P, double* __restrict__ dP) {
  const size_t q = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (q >= Rn) return;
  double a = 0.0, b = 0.0;
  for (int z = 0; z < S; ++z) {
    a += Pp[(size_t)z * Rn + q];
    b += dPp[(size_t)z * Rn + q];
  }
  P[q] = a;
  dP[q] = b;
}

// Right-hand sides of the solves: row r = P_r, row R + r = z - zbar*_r
// (zbar*_{r,i} = T[r][4 i]).
__global__ void k_vjp_rhs(const double* __restrict__ P, const double* __restrict__ z,
                          const double* __restrict__ T, int n, int R, double* __restrict__ X) {
  const size_t q = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (q >= (size_t)R * n) return;
  const size_t r = q / n, i = q % n;
  X[q] = P[q];
  X[(size_t)R * n + q] = z[i] - T[r * 4 * n + 4 * i];
}

// D[i][j] = dC(s_i - s_j)/dtheta (the theta-derivative of K22).
__global__ void k_dk22_matrix(const double* __restrict__ obs, int n, CovDev cov,
                              double* __restrict__ D) {
  const int j = blockIdx.x * 256 + threadIdx.x, i = blockIdx.y;
  if (j >= n) return;
  D[(size_t)i * n + j] = dcov_eval(cov, obs[2 * i] - obs[2 * j], obs[2 * i + 1] - obs[2 * j + 1]);
}

// The 11 products of the one-realization statistic for every r (one
// workgroup per product and realization, fixed-order reduction):
//   0 vbar.y  1 vbar.dy  2 p.cbar  3 dp.cbar  4 u.z  5 u.cbar  6 u.t_theta
//   7 u.t_sigma  8 u.t_tau  9 u.(dK22 cbar)  10 u.zbar*
__global__ void __launch_bounds__(256)
k_vjp_dots(const double* __restrict__ vbar, const double* __restrict__ Y,
           const double* __restrict__ dY, const double* __restrict__ P,
           const double* __restrict__ dP, const double* __restrict__ X,
           const double* __restrict__ z, const double* __restrict__ T,
           const double* __restrict__ Q, int M, int n, int R, double* __restrict__ out) {
  __shared__ double red[256];
  const int k = blockIdx.x, r = blockIdx.y;
  const double* u = X + (size_t)r * n;
  const double* cb = X + ((size_t)R + r) * n;
  const double* t = T + (size_t)r * 4 * n;
  const double* a;
  const double* b;
  int sb = 1, len = n;
  switch (k) {
    case 0: a = vbar + (size_t)r * M; b = Y + (size_t)r * M; len = M; break;
    case 1: a = vbar + (size_t)r * M; b = dY + (size_t)r * M; len = M; break;
    case 2: a = P + (size_t)r * n; b = cb; break;
    case 3: a = dP + (size_t)r * n; b = cb; break;
    case 4: a = u; b = z; break;
    case 5: a = u; b = cb; break;
    case 6: a = u; b = t + 1; sb = 4; break;
    case 7: a = u; b = t + 2; sb = 4; break;
    case 8: a = u; b = t + 3; sb = 4; break;
    case 9: a = u; b = Q + (size_t)r * n; break;
    default: a = u; b = t; sb = 4; break;
  }
  double acc = 0.0;
  for (int i = threadIdx.x; i < len; i += 256) acc += a[i] * b[(size_t)i * sb];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[(size_t)r * kDots + k] = red[0];
}

}  // namespace
}  // namespace cesim

using namespace cesim;

namespace {

// Arguments shared by the two entry points.
cesim_status grad_args_ok(cesim_ctx c, const double* z, double nugget, int nreal, int first_real) {
  if (nreal < 1 || first_real < 0) return CESIM_ERR_INVALID_ARG;
  if ((long)first_real + nreal > 0x7fffffffL) return CESIM_ERR_INVALID_ARG;
  if (!(std::isfinite(nugget) && nugget >= 0.0)) return CESIM_ERR_INVALID_ARG;
  if (c->nobs < 1) return CESIM_ERR_BAD_STATE;
  if (joint_active(c)) return CESIM_ERR_INVALID_ARG;   // the adjoint is of the independent sampling
  if (c->nn_active) return CESIM_ERR_INVALID_ARG;     // and of local Kriging
  for (int i = 0; i < c->nobs; ++i)
    if (!std::isfinite(z[i])) return CESIM_ERR_INVALID_ARG;
  return CESIM_OK;
}

// phi_i = sqrt(tau^2 + gamma_i): with tau^2 = 0 a station with gamma_i = 0
// (on a grid node, where gamma_i is 0 up to round-off, taken as <= 1e-12
// sigma^2) has dphi_i / dtau^2 = 1 / (2 phi_i) unbounded, so the nugget
// derivative does not exist there.  After the streams have drained.
cesim_status zero_nugget_ok(cesim_ctx c, double nugget) {
  if (nugget != 0.0) return CESIM_OK;
  const int n = c->nobs;
  std::vector<double> gm(n);
  CESIM_HIP(hipMemcpy(gm.data(), c->gamma.p, sizeof(double) * n, hipMemcpyDeviceToHost));
  for (int i = 0; i < n; ++i)
    if (!(gm[i] > 1e-12 * c->covd.sigma2)) return CESIM_ERR_INVALID_ARG;
  return CESIM_OK;
}

// The linear statistic's value and gradient (out[0..3], dz[n] on the host)
// for weights w (device, M doubles) over realizations first_real ..
// first_real + nreal - 1.
cesim_status grad_linear_core(cesim_ctx c, const double* z, double nugget, int nreal,
                              uint64_t seed, int first_real, const double* w, double* out,
                              double* dz) {
  const int n = c->nobs;
  hipStream_t s = c->stream;
  // the grid GEMM of an earlier condition() may still read the factor (aux
  // work is ordered before it), and the solves below use the stream
  CESIM_HIP(hipStreamSynchronize(c->aux));
  CESIM_HIP(hipStreamSynchronize(s));
  CESIM_TRY(zero_nugget_ok(c, nugget));
  const int M = c->grid.m1 * c->grid.m2;
  const size_t N = (size_t)c->t1 * c->t2;
  // vectors: zeta_bar 2N | ybar M | dybar M | xi_bar n | t 4n | p n | dp n | z n | X 2n | Y 2n | q n | dots
  const size_t nv = 2 * N + 2 * (size_t)M + 14 * (size_t)n + kDots;
  CESIM_TRY(c->gvec.reserve(sizeof(double) * nv));
  double* eb = c->gvec.as<double>();
  double* yb = eb + 2 * N;
  double* dyb = yb + M;
  double* xb = dyb + M;
  double* t = xb + n;
  double* p = t + 4 * (size_t)n;
  double* dp = p + n;
  double* zd = dp + n;
  double* X = zd + n;
  double* Y = X + 2 * (size_t)n;
  double* q = Y + 2 * (size_t)n;
  double* dots = q + n;
  std::vector<double> zh(z, z + n);
  CESIM_HIP(hipMemcpyAsync(zd, zh.data(), sizeof(double) * n, hipMemcpyHostToDevice, s));
  const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32), ev = (uint32_t)c->event_id;
  k_mean_pair_noise<<<(unsigned)((N / 4 + 1 + 255) / 256), 256, 0, s>>>(
      k0, k1, ev, first_real, nreal, N, reinterpret_cast<double2*>(eb));
  k_mean_obs_noise<<<(n + 255) / 256, 256, 0, s>>>(k0, k1, ev, first_real, nreal, n, xb);
  CESIM_HIP(hipGetLastError());
  CESIM_TRY(ce_grad_fields_device(c, reinterpret_cast<const double2*>(eb), yb, dyb));
  CESIM_TRY(lk_grad_device(c, nugget, yb, dyb, xb, t));
  k_cross_gemv<<<n, 256, 0, s>>>(c->obs_xy.as<double>(), c->gridd, c->covd, w, p, dp);
  k_grad_rhs<<<(n + 255) / 256, 256, 0, s>>>(p, zd, t, n, X);
  CESIM_HIP(hipGetLastError());
  // factor of A = K22 + tau^2 I (reused when it is current)
  const bool refactor = !c->chol_valid || c->chol_nugget != nugget;
  if (refactor) {
    c->chol_valid = false;
    CESIM_TRY(chol_factor_device(c, nugget, s));
  }
  CESIM_TRY(chol_solve_device(c, X, 2, s, Y));   // X = [u; cbar]
  const double* u = X;
  const double* cb = X + n;
  k_dk22_times<<<n, 256, 0, s>>>(c->obs_xy.as<double>(), n, c->covd, cb, q);
  // 0 w.ybar  1 w.dybar  2 p.cbar  3 dp.cbar  4 u.z  5 u.cbar  6 u.t_theta
  // 7 u.t_sigma  8 u.t_tau  9 u.(dK22 cbar)  10 u.zbar*
  DotList d{};
  const double* A[kDots] = {w, w, p, dp, u, u, u, u, u, u, u};
  const double* B[kDots] = {yb, dyb, cb, cb, zd, cb, t + 1, t + 2, t + 3, q, t};
  const int SB[kDots] = {1, 1, 1, 1, 1, 1, 4, 4, 4, 1, 4};
  for (int k = 0; k < kDots; ++k) {
    d.a[k] = A[k];
    d.b[k] = B[k];
    d.sb[k] = SB[k];
    d.len[k] = k < 2 ? M : n;
  }
  k_dots<<<kDots, 256, 0, s>>>(d, dots);
  CESIM_HIP(hipGetLastError());
  double h[kDots];
  CESIM_HIP(hipMemcpyAsync(h, dots, sizeof(h), hipMemcpyDeviceToHost, s));
  CESIM_HIP(hipMemcpyAsync(dz, u, sizeof(double) * n, hipMemcpyDeviceToHost, s));
  CESIM_HIP(hipStreamSynchronize(s));
  if (refactor) {
    if (c->chol_info_host[0] & 2) return CESIM_ERR_NOT_POSITIVE_DEFINITE;
    c->chol_valid = true;
    c->chol_nugget = nugget;
  }
  const double s2 = c->covd.sigma2, ub = h[4] - h[10];     // u . (z - zbar*)
  out[0] = h[0] + ub;
  out[1] = h[1] + h[3] - h[9] - h[6];
  out[2] = h[0] / (2.0 * s2) + h[2] / s2 - (ub - nugget * h[5]) / s2 - h[7];
  out[3] = -h[5] - h[8];
  return CESIM_OK;
}

// Realizations per pass of the vector-Jacobian product (bounds its arrays).
constexpr int kVjpChunk = 256;

// The vector-Jacobian product for realizations first_real .. + R - 1, all
// at once: the one-realization statistics of grad_linear_core with weights
// vbar[r], whose per-realization parts are batched -- the fields y_r and
// dy_r by two FP64 draws (with sqrt(lambda / N) and with its
// theta-derivative), the cross products K21 vbar_r and dK21 vbar_r in one
// kernel, the 2R solves in one chain, dK22 cbar_r as one GEMM.  Adds into
// acc[0..3] and dacc[n] (host).
// Node segments of the cross products: enough workgroups to fill the GPU.
int vjp_segments(cesim_ctx c, int R) {
  const int tiles = ((c->nobs + 15) / 16) * ((R + 255) / 256);
  return std::max(1, std::min(32, (1024 + tiles - 1) / tiles));
}

// Y, dY [R][M] | xi [R][n] | T [R][4n] | P, dP [R][n] | X, X2 [2R][n] | Q [R][n] |
// Pp, dPp [S][R][n] | dots [R][11]:  2 R M + (12 + 2 S) R n + 11 R doubles.
size_t vjp_chunk_doubles(cesim_ctx c, int R) {
  const size_t M = (size_t)c->grid.m1 * c->grid.m2, Rn = (size_t)R * c->nobs;
  return 2 * (size_t)R * M + (12 + 2 * (size_t)vjp_segments(c, R)) * Rn + (size_t)R * kDots;
}

// work: vjp_chunk_doubles(c, R) doubles; dk22: the n x n theta-derivative
// of K22; zd: z on the device; ds: d sqrt(lambda / N) / dtheta; slb: N
// doubles of scratch.
cesim_status vjp_chunk(cesim_ctx c, const double* zd, double nugget, int R, uint64_t seed,
                       int first_real, const double* vbar, const double* ds, double* slb,
                       const double* dk22, double* work, size_t work_doubles, double* acc,
                       double* dacc) {
  const int n = c->nobs;
  const size_t M = (size_t)c->grid.m1 * c->grid.m2, Rn = (size_t)R * n;
  hipStream_t s = c->stream;
  double* Y = work;
  double* dY = Y + (size_t)R * M;
  double* xi = dY + (size_t)R * M;
  double* T = xi + Rn;
  double* P = T + 4 * Rn;
  double* dP = P + Rn;
  double* X = dP + Rn;
  double* X2 = X + 2 * Rn;
  double* Q = X2 + 2 * Rn;
  const int S = vjp_segments(c, R);
  double* Pp = Q + Rn;
  double* dPp = Pp + (size_t)S * Rn;
  double* dots = dPp + (size_t)S * Rn;
  if ((size_t)(dots + (size_t)R * kDots - work) != vjp_chunk_doubles(c, R) ||
      vjp_chunk_doubles(c, R) > work_doubles)
    return CESIM_ERR_BAD_STATE;     // the layout, its size and the reservation disagree
  CESIM_TRY(draw_f64_spectrum_device(c, R, seed, first_real, Y, c->s64.as<double>(), slb));
  CESIM_TRY(draw_f64_spectrum_device(c, R, seed, first_real, dY, ds, slb));
  const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32), ev = (uint32_t)c->event_id;
  k_obs_noise_all<<<(unsigned)((Rn + 255) / 256), 256, 0, s>>>(k0, k1, ev, first_real, R, n, xi);
  CESIM_HIP(hipGetLastError());
  CESIM_TRY(lk_grad_device(c, nugget, Y, dY, xi, T, R));
  {
    const int seg = (int)(((M + S - 1) / S + 15) / 16 * 16);
    k_cross_adj<<<dim3((n + 15) / 16, (R + 255) / 256, S), 256, 0, s>>>(
        c->obs_xy.as<double>(), n, c->gridd, c->covd, vbar, R, seg, Pp, dPp);
    k_cross_adj_sum<<<(unsigned)((Rn + 255) / 256), 256, 0, s>>>(Pp, dPp, S, Rn, P, dP);
    CESIM_HIP(hipGetLastError());
  }
  k_vjp_rhs<<<(unsigned)((Rn + 255) / 256), 256, 0, s>>>(P, zd, T, n, R, X);
  CESIM_HIP(hipGetLastError());
  CESIM_TRY(chol_solve_device(c, X, 2 * R, s, X2));        // rows: u_r, then cbar_r
  {   // Q = Cbar dK22 (rows cbar_r; dK22 is symmetric)
    GemmArgs g;
    g.M = R; g.N = n; g.K = n; g.alpha = 1.0; g.beta = 0.0;
    g.A = X + Rn; g.sai = n; g.sak = 1;
    g.B = dk22; g.sbk = n; g.sbj = 1;
    g.C = Q; g.sci = n; g.scj = 1;
    CESIM_TRY(gemm_f64(g, false, s));
  }
  k_vjp_dots<<<dim3(kDots, R), 256, 0, s>>>(vbar, Y, dY, P, dP, X, zd, T, Q, (int)M, n, R, dots);
  CESIM_HIP(hipGetLastError());
  std::vector<double> h((size_t)R * kDots), u(Rn);
  CESIM_HIP(hipMemcpyAsync(h.data(), dots, sizeof(double) * h.size(), hipMemcpyDeviceToHost, s));
  CESIM_HIP(hipMemcpyAsync(u.data(), X, sizeof(double) * Rn, hipMemcpyDeviceToHost, s));
  CESIM_HIP(hipStreamSynchronize(s));
  const double s2 = c->covd.sigma2;
  for (int r = 0; r < R; ++r) {
    const double* e = h.data() + (size_t)r * kDots;
    const double ub = e[4] - e[10];
    acc[0] += e[0] + ub;
    acc[1] += e[1] + e[3] - e[9] - e[6];
    acc[2] += e[0] / (2.0 * s2) + e[2] / s2 - (ub - nugget * e[5]) / s2 - e[7];
    acc[3] += -e[5] - e[8];
    for (int i = 0; i < n; ++i) dacc[i] += u[(size_t)r * n + i];
  }
  return CESIM_OK;
}

}  // namespace

extern "C" cesim_status ce_grad_linear(cesim_ctx c, const double* z, double nugget, int nreal,
                                       uint64_t seed, int first_real, const void* wgt,
                                       double* out, double* dz) {
  if (!c || !z || !wgt || !out || !dz) return CESIM_ERR_INVALID_ARG;
  CESIM_TRY(grad_args_ok(c, z, nugget, nreal, first_real));
  return grad_linear_core(c, z, nugget, nreal, seed, first_real, static_cast<const double*>(wgt),
                          out, dz);
}

// The vector-Jacobian product of the conditional fields: sum over r of the
// linear statistic of realization first_real + r alone with the weights
// vbar[r] (each v_r is affine in its own noise, so the product is the sum of
// the R one-realization gradients), in chunks of kVjpChunk realizations.
extern "C" cesim_status ce_grad_vjp(cesim_ctx c, const double* z, double nugget, int nreal,
                                    uint64_t seed, int first_real, const void* vbar, double* out,
                                    double* dz) {
  if (!c || !z || !vbar || !out || !dz) return CESIM_ERR_INVALID_ARG;
  CESIM_TRY(grad_args_ok(c, z, nugget, nreal, first_real));
  const int n = c->nobs;
  const size_t M = (size_t)c->grid.m1 * c->grid.m2;
  const size_t N = (size_t)c->t1 * c->t2;
  hipStream_t s = c->stream;
  CESIM_HIP(hipStreamSynchronize(c->aux));
  CESIM_HIP(hipStreamSynchronize(s));
  CESIM_TRY(zero_nugget_ok(c, nugget));
  const int RC = std::min(nreal, kVjpChunk);
  // vjp_work: dK22 [n][n] | z [n] | the arrays of one chunk
  const size_t head = (size_t)n * n + n;
  const size_t work_doubles = vjp_chunk_doubles(c, RC);
  CESIM_TRY(c->vjp_work.reserve(sizeof(double) * (head + work_doubles)));
  double* dk22 = c->vjp_work.as<double>();
  double* zd = dk22 + (size_t)n * n;
  double* work = zd + n;
  // gwork: ds [N] | blocked-spectrum scratch [N] | complex scratch [N]
  CESIM_TRY(c->gwork.reserve(sizeof(double) * 4 * N));
  double* ds = c->gwork.as<double>();
  double* slb = ds + N;
  double2* tmp = reinterpret_cast<double2*>(slb + N);
  std::vector<double> zh(z, z + n);
  CESIM_HIP(hipMemcpyAsync(zd, zh.data(), sizeof(double) * n, hipMemcpyHostToDevice, s));
  CESIM_TRY(grad_dsqrt_device(c, ds, tmp));
  k_dk22_matrix<<<dim3((n + 255) / 256, n), 256, 0, s>>>(c->obs_xy.as<double>(), n, c->covd, dk22);
  CESIM_HIP(hipGetLastError());
  const bool refactor = !c->chol_valid || c->chol_nugget != nugget;
  if (refactor) {
    c->chol_valid = false;
    CESIM_TRY(chol_factor_device(c, nugget, s));
  }
  std::vector<double> acc(4, 0.0), dacc(n, 0.0);
  for (int r0 = 0; r0 < nreal; r0 += RC) {
    const int R = std::min(RC, nreal - r0);
    CESIM_TRY(vjp_chunk(c, zd, nugget, R, seed, first_real + r0,
                        static_cast<const double*>(vbar) + (size_t)r0 * M, ds, slb, dk22, work,
                        work_doubles, acc.data(), dacc.data()));
  }
  if (refactor) {
    if (c->chol_info_host[0] & 2) return CESIM_ERR_NOT_POSITIVE_DEFINITE;
    c->chol_valid = true;
    c->chol_nugget = nugget;
  }
  std::copy(acc.begin(), acc.end(), out);
  std::copy(dacc.begin(), dacc.end(), dz);
  return CESIM_OK;
}
