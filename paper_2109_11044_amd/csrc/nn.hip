// nn.hip -- nearest-neighbour Kriging (Section 2.2; Section 3.2): the
// observations are replaced by surrogate observations on the grid nodes of
// their (2 n_p)^2 neighbourhoods (the local-Kriging windows, overlapping
// windows merged, sites in ascending node index).  With A = K22 + tau^2 I
// of the real observations:
//   z_N       = K_N2 A^{-1} z                    (Kriging from all the data)
//   sigma_N^2 = C(0) - diag(K_N2 A^{-1} K_2N)    (its prediction error variance)
// and the sites become the context's stations: each site is its own window
// node (indicator weights), its synthetic value is y(site) + sqrt(tau^2 +
// sigma_N^2) xi, and the observation system is K_NN + tau^2 I + Sigma_N.
// condition() and ce_prediction_se then run unchanged on the surrogate
// problem (the latter gives the nearest-neighbour standard error SE_N).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "internal.hpp"

namespace cesim {
namespace {

constexpr int kMaxSites = 65535;

// K[j][i] = C(site_j - s_i)
__global__ void k_site_cross(const double* __restrict__ sxy, int ns, const double* __restrict__ obs,
                             int n, CovDev cov, double* __restrict__ K) {
  const size_t q = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (q >= (size_t)ns * n) return;
  const int j = (int)(q / n), i = (int)(q % n);
  K[q] = cov_eval(cov, sxy[2 * j] - obs[2 * i], sxy[2 * j + 1] - obs[2 * i + 1]);
}

// One workgroup per site (x = row j of K A^{-1}): sigma_N^2 = C(0) - x . k
// (clamped at 0) and z_N = x . z, fixed-order reductions.
__global__ void __launch_bounds__(256)
k_site_reduce(const double* __restrict__ K, const double* __restrict__ X,
              const double* __restrict__ z, int n, double sigma2, double* __restrict__ s2,
              double* __restrict__ zn) {
  __shared__ double red[2][256];
  const size_t o = (size_t)blockIdx.x * n;
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) {
    const double x = X[o + i];
    a += x * K[o + i];
    b += x * z[i];
  }
  red[0][threadIdx.x] = a;
  red[1][threadIdx.x] = b;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) {
      red[0][threadIdx.x] += red[0][threadIdx.x + h];
      red[1][threadIdx.x] += red[1][threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    s2[blockIdx.x] = fmax(0.0, sigma2 - red[0][0]);
    zn[blockIdx.x] = red[1][0];
  }
}

// Site j as a station with a 2 x 2 window: the weight of its own node is 1,
// the others 0, and gamma_j = sigma_N,j^2 (so phi_j^2 = tau^2 + sigma_N,j^2).
// A window that misses the site's node sets bit 2 of info.
__global__ void k_nn_install(const int* __restrict__ node, int ns, int m1,
                             const int2* __restrict__ corners, const double* __restrict__ s2,
                             double* __restrict__ W, double* __restrict__ gam,
                             int* __restrict__ info) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= ns) return;
  const int ix = node[j] % m1, iy = node[j] / m1;
  const int2 ab = corners[j];
  const int p = ix - ab.x, q = iy - ab.y;
  for (int al = 0; al < 4; ++al) W[(size_t)j * 4 + al] = 0.0;
  gam[j] = s2[j];
  if (p < 0 || p > 1 || q < 0 || q > 1) {
    atomicOr(info, 4);
    return;
  }
  W[(size_t)j * 4 + q * 2 + p] = 1.0;
}

// The ns sites (coordinates sxy on the host; node indices nd, variances s2
// on the device) become the context's stations.
cesim_status install_sites(cesim_ctx c, int ns, const double* sxy, const int* nd,
                           const double* s2) {
  hipStream_t s = c->stream;
  CESIM_TRY(offgrid_nnkrige(c, ns, sxy, 4));
  CESIM_TRY(c->nn_extra.reserve(sizeof(double) * ns));
  CESIM_HIP(hipMemcpyAsync(c->nn_extra.p, s2, sizeof(double) * ns, hipMemcpyDeviceToDevice, s));
  int* info = c->info_dev.as<int>();
  CESIM_HIP(hipMemsetAsync(info, 0, sizeof(int) * 4, s));
  k_nn_install<<<(ns + 255) / 256, 256, 0, s>>>(nd, ns, c->grid.m1, c->corners.as<int2>(),
                                                 c->nn_extra.as<double>(), c->weights.as<double>(),
                                                 c->gamma.as<double>(), info);
  CESIM_HIP(hipGetLastError());
  int hinfo[4];
  CESIM_HIP(hipMemcpyAsync(hinfo, info, sizeof(hinfo), hipMemcpyDeviceToHost, s));
  CESIM_HIP(hipStreamSynchronize(s));
  if (hinfo[0] & 4) return CESIM_ERR_BAD_STATE;
  return CESIM_OK;
}

}  // namespace
}  // namespace cesim

using namespace cesim;

extern "C" cesim_status nn_surrogate(cesim_ctx c, int nobs, const double* xy, const double* z,
                                     double nugget, int k, int capacity, double* site_xy,
                                     double* z_site, int* nsites) {
  if (!c || !xy || !z || !site_xy || !z_site || !nsites || nobs < 1 || capacity < 1)
    return CESIM_ERR_INVALID_ARG;
  if (!(std::isfinite(nugget) && nugget >= 0.0)) return CESIM_ERR_INVALID_ARG;
  for (int i = 0; i < nobs; ++i)
    if (!std::isfinite(z[i])) return CESIM_ERR_INVALID_ARG;
  *nsites = 0;
  // the observations and their windows
  CESIM_TRY(offgrid_nnkrige(c, nobs, xy, k));
  hipStream_t s = c->stream;
  const int m1 = c->grid.m1, w2 = 2 * c->npp;
  std::vector<int2> cor(nobs);
  CESIM_HIP(hipMemcpyAsync(cor.data(), c->corners.p, sizeof(int2) * nobs, hipMemcpyDeviceToHost, s));
  CESIM_HIP(hipStreamSynchronize(s));
  std::vector<int> node;
  node.reserve((size_t)nobs * k);
  for (int i = 0; i < nobs; ++i)
    for (int q = 0; q < w2; ++q)
      for (int p = 0; p < w2; ++p) node.push_back((cor[i].y + q) * m1 + cor[i].x + p);
  std::sort(node.begin(), node.end());
  node.erase(std::unique(node.begin(), node.end()), node.end());
  const int ns = (int)node.size();
  if (ns > capacity || ns > kMaxSites) return CESIM_ERR_INVALID_ARG;
  std::vector<double> sxy(2 * (size_t)ns);
  for (int j = 0; j < ns; ++j) {
    const double tx = (double)(node[j] % m1) * c->grid.dx;   // x0 + i dx, not contracted
    const double ty = (double)(node[j] / m1) * c->grid.dy;
    sxy[2 * j] = c->grid.x0 + tx;
    sxy[2 * j + 1] = c->grid.y0 + ty;
  }
  // factor of the observations' system A = K22 + tau^2 I
  c->chol_valid = false;
  CESIM_TRY(chol_factor_device(c, nugget, s));
  const size_t rows = (size_t)ns * nobs;
  CESIM_TRY(c->nn_work.reserve(sizeof(double) * (3 * rows + nobs + 4 * (size_t)ns) +
                               sizeof(int) * (size_t)ns));
  double* K = c->nn_work.as<double>();
  double* X = K + rows;
  double* Y = X + rows;
  double* zd = Y + rows;
  double* sd = zd + nobs;
  double* s2 = sd + 2 * (size_t)ns;
  double* zn = s2 + ns;
  int* nd = reinterpret_cast<int*>(zn + ns);
  CESIM_HIP(hipMemcpyAsync(zd, z, sizeof(double) * nobs, hipMemcpyHostToDevice, s));
  CESIM_HIP(hipMemcpyAsync(sd, sxy.data(), sizeof(double) * 2 * ns, hipMemcpyHostToDevice, s));
  CESIM_HIP(hipMemcpyAsync(nd, node.data(), sizeof(int) * ns, hipMemcpyHostToDevice, s));
  k_site_cross<<<(unsigned)((rows + 255) / 256), 256, 0, s>>>(sd, ns, c->obs_xy.as<double>(), nobs,
                                                              c->covd, K);
  CESIM_HIP(hipGetLastError());
  CESIM_HIP(hipMemcpyAsync(X, K, sizeof(double) * rows, hipMemcpyDeviceToDevice, s));
  CESIM_TRY(chol_solve_device(c, X, ns, s, Y));
  k_site_reduce<<<ns, 256, 0, s>>>(K, X, zd, nobs, c->covd.sigma2, s2, zn);
  CESIM_HIP(hipGetLastError());
  CESIM_HIP(hipMemcpyAsync(z_site, zn, sizeof(double) * ns, hipMemcpyDeviceToHost, s));
  CESIM_HIP(hipStreamSynchronize(s));   // also retires the staging vectors
  if (c->chol_info_host[0] & 2) return CESIM_ERR_NOT_POSITIVE_DEFINITE;
  std::copy(sxy.begin(), sxy.end(), site_xy);
  // the sites become the stations; a failure from here on leaves none, so
  // that condition() cannot run the sites as plain local-Kriging stations
  const cesim_status ist = install_sites(c, ns, sxy.data(), nd, s2);
  if (ist != CESIM_OK) {
    c->nobs = 0;
    return ist;
  }
  c->nboxes = 0;                        // every site is its own grid node
  c->max_box = 0;
  c->nn_active = true;
  c->chol_valid = false;
  c->yhat_valid = false;
  *nsites = ns;
  return CESIM_OK;
}
