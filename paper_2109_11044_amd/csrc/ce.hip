// ce.hip -- circulant-embedding setup and the batched unconditional draw.
//
// Setup (Section 1; Section 2.1 item (a)): the torus base
//   c[q2][q1] = C(w(q1) dx, w(q2) dy),  w(q) = q (q <= T/2) else q - T,
// Nyquist lines averaged over the sign of their lag component, its 2D FFT in
// FP64, the eigenvalue checks in FP64, and sqrt(lambda) / (t1 t2) kept in
// FP64 and FP32.
//
// Draw (step 2 of Section 2): per pair of realizations (2p, 2p+1)
//   pass 1: Philox noise eps_{2p} + i eps_{2p+1} -> forward FFT of every
//           torus row (x) in LDS -> pair buffer;
//   pass 2: per panel of columns: forward FFT along y, multiply by
//           sqrt(lambda)/N, inverse FFT along y; only the m2 rows the crop
//           keeps are written back;
//   pass 3: per kept row: inverse FFT along x; the first m1 outputs give
//           field 2p (real part) and field 2p+1 (imaginary part).
// Because lambda is real and even the map eps -> field is real, so the two
// realizations in one complex transform do not mix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <mutex>
#include <vector>

#include "internal.hpp"
#include "fft_pow2.hpp"

namespace cesim {

// ------------------------------------------------------------------ kernels

__global__ void k_twiddles(int T, double2* tw64, float2* tw32) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= T) return;
  double s, c;
  sincospi(-2.0 * (double)t / (double)T, &s, &c);
  tw64[t] = {c, s};
  tw32[t] = {(float)c, (float)s};
}

__device__ inline int wrapped_lag(int q, int T) { return q <= T / 2 ? q : q - T; }

// DTH: the theta-derivative of the base instead (same lags, same averaging).
template <bool DTH>
__global__ void k_torus_base(CovDev cov, double dx, double dy, int t1, int t2, double2* out) {
  const int q1 = blockIdx.x * blockDim.x + threadIdx.x;
  const int q2 = blockIdx.y;
  if (q1 >= t1) return;
  const double hx = (double)wrapped_lag(q1, t1) * dx;
  const double hy = (double)wrapped_lag(q2, t2) * dy;
  const bool nyq1 = (t1 % 2 == 0) && (2 * q1 == t1);
  const bool nyq2 = (t2 % 2 == 0) && (2 * q2 == t2);
  auto f = [&](double a, double b) { return DTH ? dcov_eval(cov, a, b) : cov_eval(cov, a, b); };
  double c;
  if (nyq1) {
    c = 0.5 * (f(hx, hy) + f(-hx, hy));
  } else if (nyq2) {
    c = 0.5 * (f(hx, hy) + f(hx, -hy));
  } else {
    c = f(hx, hy);
  }
  out[(size_t)q2 * t1 + q1] = {c, 0.0};
}

// Copies the twiddle table into LDS after the data (when it fits) so that
// the stages read it without global-memory latency; the caller's barrier
// after loading the data also covers this copy.
template <typename real, int NTHR>
__device__ inline const cpx<real>* stage_twiddles(cpx<real>* dst, const cpx<real>* __restrict__ tw,
                                                 int T, bool tw_lds) {
  if (!tw_lds) return tw;
  for (int t = threadIdx.x; t < T; t += NTHR) dst[t] = tw[t];
  return dst;
}

// Absolute pair of workgroup row p of a draw launch: pairs are (2P, 2P + 1)
// in absolute realization numbers, so a call starting at an odd realization
// begins with the second member of a pair.  Returns realization 2P, or -1
// for a spare pair beyond the call (graphs replayed at an offset of either
// parity are captured with one spare pair).
__device__ __forceinline__ int pair_first_real(const NoiseKey& key, int nreal, int pair0, int p) {
  const int first = key.base();
  const int r0 = 2 * ((first >> 1) + pair0 + p);
  return r0 < first + nreal ? r0 : -1;
}

// Four normals of Philox block blk for each member of the pair (2P, 2P + 1).
template <typename real>
__device__ __forceinline__ void pair_normals(const NoiseKey& key, uint32_t blk, int r0, real za[4],
                                             real zb[4]) {
  if constexpr (sizeof(real) == 8) {
    normals4_f64(key.k0, key.k1, blk, (uint32_t)r0, key.event, 0u, za);
    normals4_f64(key.k0, key.k1, blk, (uint32_t)(r0 + 1), key.event, 0u, zb);
  } else {
    normals4_f32(key.k0, key.k1, blk, (uint32_t)r0, key.event, 0u, za);
    normals4_f32(key.k0, key.k1, blk, (uint32_t)(r0 + 1), key.event, 0u, zb);
  }
}

// Crop of one transformed row j of pair (2P, 2P + 1): the first m1 entries
// give realization 2P (real part) and 2P + 1 (imaginary part), each written
// when it belongs to the call (fields[r - first]).
template <typename real>
struct CropRow {
  real* re = nullptr;
  real* im = nullptr;
  __device__ CropRow(real* fields, const NoiseKey& key, int nreal, int r0, int m1, int m2, int j) {
    const long f0 = (long)r0 - key.base();          // -1 .. nreal - 1
    const size_t M = (size_t)m1 * m2;
    if (f0 >= 0) re = fields + (size_t)f0 * M + (size_t)j * m1;
    if (f0 + 1 < nreal) im = fields + (size_t)(f0 + 1) * M + (size_t)j * m1;
  }
  template <typename C>
  __device__ __forceinline__ void put(int x, C v) const {
    if (re) re[x] = v.x;
    if (im) im[x] = v.y;
  }
};

// Forward FFT of nb rows per workgroup, in place (the setup's 2D FFT and
// the gradient's draw of the mean noise).
template <typename real, int NTHR, int E>
__global__ void __launch_bounds__(NTHR)
k_rows_fwd(cpx<real>* __restrict__ buf, int t1, int t2, int nb, Plan plan,
           const cpx<real>* __restrict__ tw, bool tw_lds) {
  extern __shared__ __align__(16) unsigned char smem[];
  cpx<real>* lds = reinterpret_cast<cpx<real>*>(smem);
  const int j0 = blockIdx.x * nb;
  const int nr = min(nb, t2 - j0);
  cpx<real>* base = buf + (size_t)j0 * t1;
  const cpx<real>* twl = stage_twiddles<real, NTHR>(lds + nb * t1, tw, t1, tw_lds);
  for (int e = threadIdx.x; e < nr * t1; e += NTHR) lds[e] = base[e];
  __syncthreads();
  fft_lds<false, NTHR, E, false, real>(lds, plan, nr, 1, t1, twl);
  for (int e = threadIdx.x; e < nr * t1; e += NTHR) base[e] = lds[e];
}

// Forward FFT of a panel of cp columns, in place, all rows.
template <typename real, int NTHR, int E>
__global__ void __launch_bounds__(NTHR)
k_cols(cpx<real>* __restrict__ buf, int t1, int t2, int cp, Plan plan,
       const cpx<real>* __restrict__ tw, bool tw_lds) {
  extern __shared__ __align__(16) unsigned char smem[];
  cpx<real>* lds = reinterpret_cast<cpx<real>*>(smem);
  const cpx<real>* twl = stage_twiddles<real, NTHR>(lds + cp * t2, tw, t2, tw_lds);
  const int c0 = blockIdx.x * cp;
  const int cw = min(cp, t1 - c0);
  cpx<real>* base = buf + c0;
  for (int e = threadIdx.x; e < t2 * cp; e += NTHR) {
    const int row = e / cp, c = e - row * cp;
    lds[e] = c < cw ? base[(size_t)row * t1 + c] : cpx<real>{0, 0};
  }
  __syncthreads();
  fft_lds<false, NTHR, E, true, real>(lds, plan, cp, cp, 1, twl);
  for (int e = threadIdx.x; e < t2 * cp; e += NTHR) {
    const int row = e / cp, c = e - row * cp;
    if (c < cw) base[(size_t)row * t1 + c] = lds[e];
  }
}

// Draw pass A, any torus: a panel of cp columns of pair p.  The pair noise
// eps_{2P} + i eps_{2P+1} (element q = j t1 + i: Philox block q / 4, word
// q % 4) times s = sqrt(lambda / N), forward FFT along y, rows < m2 stored
// as buf[p][row][col] (row stride t1).
template <typename real, int NTHR, int E>
__global__ void __launch_bounds__(NTHR)
k_cols_noise(cpx<real>* __restrict__ buf, int t1, int t2, int cp, int m2, Plan plan,
             const cpx<real>* __restrict__ tw, bool tw_lds, const real* __restrict__ s,
             NoiseKey key, int nreal, int pair0) {
  extern __shared__ __align__(16) unsigned char smem[];
  cpx<real>* lds = reinterpret_cast<cpx<real>*>(smem);
  const int p = blockIdx.y;
  const int r0 = pair_first_real(key, nreal, pair0, p);
  if (r0 < 0) return;
  const cpx<real>* twl = stage_twiddles<real, NTHR>(lds + cp * t2, tw, t2, tw_lds);
  const int c0 = blockIdx.x * cp;
  const int cw = min(cp, t1 - c0);
  // blocks covering elements j t1 + c0 .. j t1 + c0 + cw - 1 of each row
  const int bpr = (cw + 3) / 4 + 1;
  for (int e = threadIdx.x; e < t2 * bpr; e += NTHR) {
    const int row = e / bpr, g = e - row * bpr;
    const long q_lo = (long)row * t1 + c0;
    const long b = (q_lo >> 2) + g;
    if (4 * b >= q_lo + cw) continue;
    real za[4], zb[4];
    pair_normals<real>(key, (uint32_t)b, r0, za, zb);
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      const long q = 4 * b + w;
      if (q >= q_lo && q < q_lo + cw) {
        const int c = (int)(q - q_lo);
        const real m = s[q];
        lds[row * cp + c] = {za[w] * m, zb[w] * m};
      }
    }
  }
  for (int e = threadIdx.x; e < t2 * cp; e += NTHR)     // ragged last panel
    if (e % cp >= cw) lds[e] = cpx<real>{0, 0};
  __syncthreads();
  fft_lds<false, NTHR, E, true, real>(lds, plan, cp, cp, 1, twl);
  cpx<real>* out = buf + (size_t)p * m2 * t1 + c0;
  for (int e = threadIdx.x; e < m2 * cp; e += NTHR) {
    const int row = e / cp, c = e - row * cp;
    if (c < cw) out[(size_t)row * t1 + c] = lds[e];
  }
}

// Draw pass B, any torus: forward FFT along x of nb kept rows (y < m2) of
// pair p and the crop into realizations 2P (real part) and 2P + 1
// (imaginary part).
template <typename real, int NTHR, int E>
__global__ void __launch_bounds__(NTHR)
k_rows_crop(const cpx<real>* __restrict__ buf, real* __restrict__ fields, int t1, int m1, int m2,
            int nb, Plan plan, const cpx<real>* __restrict__ tw, bool tw_lds, NoiseKey key,
            int nreal, int pair0) {
  extern __shared__ __align__(16) unsigned char smem[];
  cpx<real>* lds = reinterpret_cast<cpx<real>*>(smem);
  const int p = blockIdx.y;
  const int r0 = pair_first_real(key, nreal, pair0, p);
  if (r0 < 0) return;
  const cpx<real>* twl = stage_twiddles<real, NTHR>(lds + nb * t1, tw, t1, tw_lds);
  const int j0 = blockIdx.x * nb;
  const int nr = min(nb, m2 - j0);
  const cpx<real>* base = buf + ((size_t)p * m2 + j0) * t1;
  for (int e = threadIdx.x; e < nr * t1; e += NTHR) lds[e] = base[e];
  __syncthreads();
  fft_lds<false, NTHR, E, false, real>(lds, plan, nr, 1, t1, twl);
  for (int e = threadIdx.x; e < nr * m1; e += NTHR) {
    const int row = e / m1, x = e - row * m1;
    const CropRow<real> cr(fields, key, nreal, r0, m1, m2, j0 + row);
    cr.put(x, lds[row * t1 + x]);
  }
}

// ------------------------------------------- power-of-two draw kernels
// The same two passes with the transform length fixed at compile time and
// the data held in registers (see fft_pow2.hpp).

// Pass A: CP columns per workgroup.  The pair noise of the panel goes into
// LDS (a Philox block holds 4 adjacent columns of one row), each element is
// scaled by s = sqrt(lambda / N) read from the copy blocked by 8 columns (a
// wave reads 8 rows of 8 columns contiguously), the forward FFT along y runs
// in registers and rows < m2 are stored as buf[p][row][col].
template <typename real, int T>
__global__ void __launch_bounds__((P2Cols<real, T>::NTHR))
k_p2_cols_noise(cpx<real>* __restrict__ buf, int m2, const cpx<real>* __restrict__ tw,
                const real* __restrict__ slb, int lcp, NoiseKey key, int nreal, int pair0) {
  using C = cpx<real>;
  using G = P2Cols<real, T>;
  extern __shared__ __align__(16) unsigned char smem[];
  C* lds = reinterpret_cast<C*>(smem);
  const int p = blockIdx.y;
  const int r0 = pair_first_real(key, nreal, pair0, p);
  if (r0 < 0) return;
  const int cp = 1 << lcp;
  // Workgroups are dealt to the 8 XCDs round-robin; when the panel count is
  // a multiple of 8, panels are renumbered so that one XCD takes adjacent
  // panels in turn and the halves of each cache line meet in its L2.
  int panel = blockIdx.x;
  if ((gridDim.x & 7) == 0) panel = (blockIdx.x & 7) * (gridDim.x >> 3) + (blockIdx.x >> 3);
  const int col0 = panel * cp;
  const int bpr = cp >= 4 ? cp >> 2 : 1;             // Philox blocks per row of the panel
  const int i00 = col0 & ~3;
  for (int e = threadIdx.x; e < T * bpr; e += blockDim.x) {
    const int row = e >> (lcp >= 2 ? lcp - 2 : 0);
    const int i0 = i00 + 4 * (e - row * bpr);
    real za[4], zb[4];
    pair_normals<real>(key, (uint32_t)(((long)row * T + i0) >> 2), r0, za, zb);
    const int pr = (row + (row >> 4)) << lcp;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      const int c = i0 + w - col0;
      if (c >= 0 && c < cp) lds[pr + c] = C{za[w], zb[w]};
    }
  }
  __syncthreads();
  const int c = threadIdx.x & (cp - 1), hb = threadIdx.x >> lcp;
  const int col = col0 + c;
  const ColLds<C> cl{lds, c, lcp};
  C x[G::E];
#pragma unroll
  for (int h = 0; h < G::E; ++h) {
    const int row = hb + G::S * h;
    const C v = cl.load(row);
    const real m = slb[((size_t)(col >> 3) * T + row) * 8 + (col & 7)];
    x[h] = {v.x * m, v.y * m};
  }
  p2_fft<real, T, false>(x, hb, tw, cl);
  C* colp = buf + (size_t)p * m2 * T + col;
#pragma unroll
  for (int h = 0; h < G::E; ++h) {
    const int row = hb + G::S * h;
    if (row < m2) colp[(size_t)row * T] = x[h];
  }
}

// Pass B: ROWS kept rows per workgroup: forward row FFT and the crop into
// realizations 2P (real part) and 2P + 1 (imaginary part).
template <typename real, int T>
__global__ void __launch_bounds__(P2Rows<T>::NTHR)
k_p2_rows_crop(const cpx<real>* __restrict__ buf, real* __restrict__ fields, int m1, int m2,
               const cpx<real>* __restrict__ tw, NoiseKey key, int nreal, int pair0) {
  using C = cpx<real>;
  using G = P2Rows<T>;
  extern __shared__ __align__(16) unsigned char smem[];
  C* lds = reinterpret_cast<C*>(smem);
  const int p = blockIdx.y;
  const int r0 = pair_first_real(key, nreal, pair0, p);
  if (r0 < 0) return;
  const int b = threadIdx.x / G::S, hb = threadIdx.x % G::S;
  const int j = blockIdx.x * (blockDim.x / G::S) + b;
  const bool ok = j < m2;
  const C* in = buf + ((size_t)p * m2 + (ok ? j : 0)) * T;
  C x[G::E];
#pragma unroll
  for (int h = 0; h < G::E; ++h) x[h] = ok ? in[hb + G::S * h] : C{0, 0};
  const RowLds<C> rl{lds + b * G::LD};
  p2_fft<real, T, false>(x, hb, tw, rl);
  if (!ok) return;
  const CropRow<real> cr(fields, key, nreal, r0, m1, m2, j);
#pragma unroll
  for (int h = 0; h < G::E; ++h) {
    const int xcol = hb + G::S * h;
    if (xcol < m1) cr.put(xcol, x[h]);
  }
}

// Eigenvalue statistics: min, max, sum of Re and max |Im|.
__global__ void k_eig_partial(const double2* lam, size_t N, double* part) {
  __shared__ double smin[256], smax[256], ssum[256], sim[256];
  double mn = INFINITY, mx = -INFINITY, sm = 0.0, im = 0.0;
  for (size_t q = blockIdx.x * 256 + threadIdx.x; q < N; q += (size_t)gridDim.x * 256) {
    const double2 v = lam[q];
    mn = fmin(mn, v.x);
    mx = fmax(mx, v.x);
    sm += v.x;
    im = fmax(im, fabs(v.y));
  }
  smin[threadIdx.x] = mn; smax[threadIdx.x] = mx; ssum[threadIdx.x] = sm; sim[threadIdx.x] = im;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) {
      smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + h]);
      smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + h]);
      ssum[threadIdx.x] += ssum[threadIdx.x + h];
      sim[threadIdx.x] = fmax(sim[threadIdx.x], sim[threadIdx.x + h]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[4 * blockIdx.x + 0] = smin[0];
    part[4 * blockIdx.x + 1] = smax[0];
    part[4 * blockIdx.x + 2] = ssum[0];
    part[4 * blockIdx.x + 3] = sim[0];
  }
}

__global__ void __launch_bounds__(512) k_eig_final(const double* part, int nparts, double* out) {
  __shared__ double smin[512], smax[512], ssum[512], sim[512];
  const int t = threadIdx.x;
  const bool ok = t < nparts;
  smin[t] = ok ? part[4 * t] : INFINITY;
  smax[t] = ok ? part[4 * t + 1] : -INFINITY;
  ssum[t] = ok ? part[4 * t + 2] : 0.0;
  sim[t] = ok ? part[4 * t + 3] : 0.0;
  __syncthreads();
  for (int h = 256; h > 0; h >>= 1) {
    if (t < h) {
      smin[t] = fmin(smin[t], smin[t + h]);
      smax[t] = fmax(smax[t], smax[t + h]);
      ssum[t] += ssum[t + h];
      sim[t] = fmax(sim[t], sim[t + h]);
    }
    __syncthreads();
  }
  if (t == 0) {
    out[0] = smin[0]; out[1] = smax[0]; out[2] = ssum[0]; out[3] = sim[0];
  }
}

// s = sqrt(lambda / N), the multiplier of the draw (lambda clamped at 0).
__global__ void k_sqrt_lambda(const double2* lam, size_t N, double rsqrt_n, double* s64,
                              float* s32) {
  const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= N) return;
  const double v = sqrt(fmax(lam[q].x, 0.0)) * rsqrt_n;
  s64[q] = v;
  if (s32) s32[q] = (float)v;
}

// sqrt(lambda / N) of the register draw path, in the path's precision and
// blocked by 8 columns: element (row r, column q) at ((q / 8) t2 + r) 8 + q % 8
// (t1 is a multiple of 8 on that path).
template <typename real>
__global__ void k_block_lambda(const double* __restrict__ s64, int t1, int t2,
                               real* __restrict__ out) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)t1 * t2) return;
  const int r = (int)(e / t1), q = (int)(e % t1);
  out[((size_t)(q >> 3) * t2 + r) * 8 + (q & 7)] = (real)s64[e];
}

// ------------------------------------------------------------------- host

cesim_status make_plan(int T, Plan& p) {
  p.T = T;
  p.nst = 0;
  int n = T;
  int twos = 0;
  while (n % 2 == 0) { n /= 2; ++twos; }
  while (twos >= 3 && !(twos == 4)) {       // prefer 8s, finish 2^4 as 4 * 4
    p.rad[p.nst++] = 8;
    twos -= 3;
  }
  while (twos >= 2) { p.rad[p.nst++] = 4; twos -= 2; }
  if (twos == 1) p.rad[p.nst++] = 2;
  while (n % 3 == 0) { p.rad[p.nst++] = 3; n /= 3; }
  while (n % 5 == 0) { p.rad[p.nst++] = 5; n /= 5; }
  if (n != 1 || p.nst > 16) return CESIM_ERR_INVALID_ARG;
  return CESIM_OK;
}

cesim_status make_twiddles(int T, DevBuf& tw64, DevBuf& tw32, hipStream_t s) {
  CESIM_TRY(tw64.reserve(sizeof(double2) * T));
  CESIM_TRY(tw32.reserve(sizeof(float2) * T));
  k_twiddles<<<(T + 255) / 256, 256, 0, s>>>(T, tw64.as<double2>(), tw32.as<float2>());
  CESIM_HIP(hipGetLastError());
  return CESIM_OK;
}

namespace {

constexpr int kRowThreads = 256;
constexpr int kColThreads = 512;
constexpr size_t kLdsTotal = 160 * 1024;

// Rows per workgroup, elements per thread and whether the twiddle table
// sits in LDS, for the row kernels.
template <typename real>
void row_config(int T, int& nb, int& E, bool& tw_lds, size_t& lds) {
  const size_t cs = sizeof(cpx<real>);
  nb = std::max(1, 4096 / T);
  while (nb > 1 && (size_t)nb * T * cs > kLdsTotal / 2) --nb;
  tw_lds = (size_t)(nb + 1) * T * cs <= kLdsTotal;
  lds = (size_t)(nb + (tw_lds ? 1 : 0)) * T * cs;
  const int el = nb * T;
  E = el <= 16 * kRowThreads ? 16 : 32;
}

template <typename real>
void col_config(int T, int t1, int& cp, int& E, bool& tw_lds, size_t& lds) {
  const size_t cs = sizeof(cpx<real>);
  tw_lds = (size_t)2 * T * cs <= kLdsTotal;          // table and at least one column
  const size_t cap = (kLdsTotal - (tw_lds ? T * cs : 0)) / cs;
  cp = std::max(1, (int)std::min<size_t>(16, cap / T));
  int c = 1;
  while (c * 2 <= cp) c *= 2;
  cp = std::min(c, std::max(1, t1));
  lds = ((size_t)cp * T + (tw_lds ? T : 0)) * cs;
  const int el = cp * T;
  E = el <= 4 * kColThreads ? 4 : el <= 8 * kColThreads ? 8 : el <= 16 * kColThreads ? 16 : 32;
}

template <typename K>
void allow_lds(K kernel, size_t bytes) {
  if (bytes > 64 * 1024)
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

// Forward 2D FFT of one t2 x t1 complex array in place (rows, then columns).
template <typename real>
cesim_status fft2_forward(cpx<real>* buf, int t1, int t2, const Plan& p1, const Plan& p2,
                          const cpx<real>* tw1, const cpx<real>* tw2, hipStream_t s) {
  int nb, E, cp;
  bool twl;
  size_t lds;
  row_config<real>(t1, nb, E, twl, lds);
  {
    const dim3 grid((t2 + nb - 1) / nb);
    auto k = E == 16 ? k_rows_fwd<real, kRowThreads, 16> : k_rows_fwd<real, kRowThreads, 32>;
    allow_lds(k, lds);
    k<<<grid, kRowThreads, lds, s>>>(buf, t1, t2, nb, p1, tw1, twl);
    CESIM_HIP(hipGetLastError());
  }
  col_config<real>(t2, t1, cp, E, twl, lds);
  {
    const dim3 grid((t1 + cp - 1) / cp);
    auto k = E == 4 ? k_cols<real, kColThreads, 4>
           : E == 8 ? k_cols<real, kColThreads, 8>
           : E == 16 ? k_cols<real, kColThreads, 16> : k_cols<real, kColThreads, 32>;
    allow_lds(k, lds);
    k<<<grid, kColThreads, lds, s>>>(buf, t1, t2, cp, p2, tw2, twl);
    CESIM_HIP(hipGetLastError());
  }
  return CESIM_OK;
}

// Draw pass A on any torus (LDS Stockham).
template <typename real>
cesim_status launch_cols_noise(cpx<real>* buf, int t1, int t2, int m2, int npairs,
                               const Plan& plan, const cpx<real>* tw, const real* s,
                               const NoiseKey& key, int nreal, int pair0, hipStream_t st) {
  int cp, E;
  bool twl;
  size_t lds;
  col_config<real>(t2, t1, cp, E, twl, lds);
  const dim3 grid((t1 + cp - 1) / cp, npairs);
  auto k = E == 4 ? k_cols_noise<real, kColThreads, 4>
         : E == 8 ? k_cols_noise<real, kColThreads, 8>
         : E == 16 ? k_cols_noise<real, kColThreads, 16> : k_cols_noise<real, kColThreads, 32>;
  allow_lds(k, lds);
  k<<<grid, kColThreads, lds, st>>>(buf, t1, t2, cp, m2, plan, tw, twl, s, key, nreal, pair0);
  CESIM_HIP(hipGetLastError());
  return CESIM_OK;
}

// Draw pass B on any torus (LDS Stockham).
template <typename real>
cesim_status launch_rows_crop(const cpx<real>* buf, real* fields, int t1, int m1, int m2,
                              int npairs, const Plan& plan, const cpx<real>* tw,
                              const NoiseKey& key, int nreal, int pair0, hipStream_t s) {
  int nb, E;
  bool twl;
  size_t lds;
  row_config<real>(t1, nb, E, twl, lds);
  const dim3 grid((m2 + nb - 1) / nb, npairs);
  auto k = E == 16 ? k_rows_crop<real, kRowThreads, 16> : k_rows_crop<real, kRowThreads, 32>;
  allow_lds(k, lds);
  k<<<grid, kRowThreads, lds, s>>>(buf, fields, t1, m1, m2, nb, plan, tw, twl, key, nreal, pair0);
  CESIM_HIP(hipGetLastError());
  return CESIM_OK;
}

}  // namespace

cesim_status ce_setup_device(cesim_ctx c, int t1, int t2, bool& accepted) {
  hipStream_t s = c->stream;
  Plan p1, p2;
  CESIM_TRY(make_plan(t1, p1));
  CESIM_TRY(make_plan(t2, p2));
  c->tt.p1 = p1;
  c->tt.p2 = p2;
  CESIM_TRY(make_twiddles(t1, c->tt.tw1_64, c->tt.tw1_32, s));
  CESIM_TRY(make_twiddles(t2, c->tt.tw2_64, c->tt.tw2_32, s));
  const size_t N = (size_t)t1 * t2;
  CESIM_TRY(c->work.reserve(sizeof(double2) * N));
  double2* buf = c->work.as<double2>();
  int tr = c->timer.begin(ST_SETUP_BASE, s);
  k_torus_base<false><<<dim3((t1 + 255) / 256, t2), 256, 0, s>>>(c->covd, c->grid.dx, c->grid.dy,
                                                                 t1, t2, buf);
  CESIM_HIP(hipGetLastError());
  c->timer.end(tr, s);
  tr = c->timer.begin(ST_SETUP_FFT, s);
  CESIM_TRY(fft2_forward<double>(buf, t1, t2, p1, p2, c->tt.tw1_64.as<double2>(),
                                 c->tt.tw2_64.as<double2>(), s));
  c->timer.end(tr, s);
  const int nparts = 512;
  CESIM_TRY(c->scratch.reserve(sizeof(double) * (4 * nparts + 8)));
  double* part = c->scratch.as<double>();
  tr = c->timer.begin(ST_SETUP_EIG, s);
  k_eig_partial<<<nparts, 256, 0, s>>>(buf, N, part);
  k_eig_final<<<1, 512, 0, s>>>(part, nparts, part + 4 * nparts);
  CESIM_HIP(hipGetLastError());
  c->timer.end(tr, s);
  double st[4];
  CESIM_HIP(hipMemcpyAsync(st, part + 4 * nparts, sizeof(st), hipMemcpyDeviceToHost, s));
  CESIM_HIP(hipStreamSynchronize(s));
  c->lam_min = st[0];
  c->lam_max = st[1];
  c->lam_sum = st[2];
  c->max_imag = st[3];
  // The spectrum of a valid embedding: non-negative up to round-off
  // (lambda_min >= -1e-12 lambda_max), real (the base is even, so any
  // imaginary part is round-off: max |Im| <= 1e-12 lambda_max), and with the
  // trace identity sum(lambda) = N c[0][0] = N C(0) to 1e-9 relative.
  const double trace = (double)N * c->covd.sigma2;
  accepted = std::isfinite(st[0]) && std::isfinite(st[1]) && std::isfinite(st[2]) &&
             std::isfinite(st[3]) && st[0] >= -1e-12 * st[1] && st[3] <= 1e-12 * st[1] &&
             std::fabs(st[2] - trace) <= 1e-9 * trace;
  if (!accepted) return CESIM_OK;
  CESIM_TRY(c->s64.reserve(sizeof(double) * N));
  float* s32 = nullptr;
  if (c->prec == CESIM_PREC_MIXED) {
    CESIM_TRY(c->s32.reserve(sizeof(float) * N));
    s32 = c->s32.as<float>();
  }
  tr = c->timer.begin(ST_SETUP_EIG, s);
  k_sqrt_lambda<<<(unsigned)((N + 255) / 256), 256, 0, s>>>(buf, N, 1.0 / std::sqrt((double)N),
                                                            c->s64.as<double>(), s32);
  CESIM_HIP(hipGetLastError());
  if (register_draw_torus(t1, t2)) {       // c->t1, c->t2 are set after acceptance
    const unsigned nb = (unsigned)((N + 255) / 256);
    if (c->prec == CESIM_PREC_MIXED) {
      CESIM_TRY(c->slb.reserve(sizeof(float) * N));
      k_block_lambda<float><<<nb, 256, 0, s>>>(c->s64.as<double>(), t1, t2, c->slb.as<float>());
    } else {
      CESIM_TRY(c->slb.reserve(sizeof(double) * N));
      k_block_lambda<double><<<nb, 256, 0, s>>>(c->s64.as<double>(), t1, t2, c->slb.as<double>());
    }
    CESIM_HIP(hipGetLastError());
  }
  c->timer.end(tr, s);
  return CESIM_OK;
}

namespace {

// Tile shape of the register path: log2 of the columns per workgroup of
// pass A and the rows per workgroup of pass B, clamped to each kernel's
// maximum (results do not depend on it).
template <typename real, int T1, int T2>
DrawShape clamp_shape(DrawShape d) {
  using GR = P2Rows<T1>;
  using GC = P2Cols<real, T2>;
  int v = GR::ROWS;
  if (d.rows > 0) while (v > 1 && v > d.rows) v >>= 1;
  d.rows = v;
  const int lmax = ilog2c(GC::CP);
  d.lcp = (d.lcp < 0 || d.lcp > lmax) ? lmax : d.lcp;
  return d;
}

template <typename real, int T1, int T2>
cesim_status draw_chunk_p2(cpx<real>* buf, real* fields, int m1, int m2, int np, const cpx<real>* tw1,
                           const cpx<real>* tw2, const real* slb, const NoiseKey& key, int nreal,
                           int pair0, const DrawShape& shape, StageTimer& tm, hipStream_t s) {
  using GR = P2Rows<T1>;
  using GC = P2Cols<real, T2>;
  const DrawShape d = clamp_shape<real, T1, T2>(shape);
  const int cp = 1 << d.lcp;
  const size_t lc = sizeof(cpx<real>) * cp * GC::LD;
  const size_t lr = sizeof(cpx<real>) * d.rows * GR::LD;
  int tr = tm.begin(ST_DRAW_PASS_A, s);
  {
    auto k = k_p2_cols_noise<real, T2>;
    allow_lds(k, sizeof(cpx<real>) * GC::CP * GC::LD);
    k<<<dim3((T1 + cp - 1) / cp, np), cp * GC::S, lc, s>>>(buf, m2, tw2, slb, d.lcp, key, nreal,
                                                           pair0);
    CESIM_HIP(hipGetLastError());
  }
  tm.end(tr, s);
  tr = tm.begin(ST_DRAW_PASS_B, s);
  {
    auto k = k_p2_rows_crop<real, T1>;
    allow_lds(k, sizeof(cpx<real>) * GR::ROWS * GR::LD);
    k<<<dim3((m2 + d.rows - 1) / d.rows, np), d.rows * GR::S, lr, s>>>(buf, fields, m1, m2, tw1,
                                                                       key, nreal, pair0);
    CESIM_HIP(hipGetLastError());
  }
  tm.end(tr, s);
  return CESIM_OK;
}

// Square tori of 2^a from 128 to 8192 and of 3 * 2^a from 384 to 6144 take
// the register path (16 or 24 elements per thread).
template <typename real>
bool draw_chunk_pow2(int t1, int t2, cpx<real>* buf, real* fields, int m1, int m2, int np,
                     const cpx<real>* tw1, const cpx<real>* tw2, const real* slb,
                     const NoiseKey& key, int nreal, int pair0, const DrawShape& shape,
                     StageTimer& tm, hipStream_t s, cesim_status& st) {
  if (t1 != t2) return false;
  switch (t1) {
#define CESIM_P2(TT)                                                                        \
  case TT:                                                                                  \
    st = draw_chunk_p2<real, TT, TT>(buf, fields, m1, m2, np, tw1, tw2, slb, key, nreal, pair0, \
                                     shape, tm, s);                                         \
    return true;
    CESIM_P2(128) CESIM_P2(256) CESIM_P2(512) CESIM_P2(1024) CESIM_P2(2048) CESIM_P2(4096)
    CESIM_P2(8192)
    default: break;
  }
  switch (t1) {
    CESIM_P2(384) CESIM_P2(768) CESIM_P2(1536) CESIM_P2(3072) CESIM_P2(6144)
    default: break;
  }
#undef CESIM_P2
  return false;
}

template <typename real>
cesim_status draw_typed(cesim_ctx c, int nreal, uint64_t seed, int first_real, real* fields,
                        const cpx<real>* tw1, const cpx<real>* tw2, const real* sl,
                        const real* slb, void* work, size_t work_bytes) {
  hipStream_t s = c->stream;
  const int t1 = c->t1, t2 = c->t2, m1 = c->grid.m1, m2 = c->grid.m2;
  // in this draw's precision (an FP64 draw also runs on a mixed context)
  const size_t pair_bytes = sizeof(cpx<real>) * (size_t)t1 * m2;
  const int npairs = draw_npairs(c, nreal, first_real);
  int chunk = draw_chunk_pairs(c, nreal, first_real);
  cpx<real>* buf;
  if (work) {                       // pair buffers lent by the caller
    chunk = std::min<size_t>(chunk, work_bytes / pair_bytes);
    if (chunk < 1) return CESIM_ERR_INVALID_ARG;
    buf = static_cast<cpx<real>*>(work);
  } else {
    CESIM_TRY(c->work.reserve(pair_bytes * chunk));
    buf = c->work.as<cpx<real>>();
  }
  const NoiseKey key{(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32), first_real,
                     c->event_id, c->roff};
  const DrawShape shape = draw_shape(c);
  if (register_draw_torus(t1, t2) && slb == nullptr) return CESIM_ERR_BAD_STATE;
  for (int pair0 = 0; pair0 < npairs; pair0 += chunk) {
    const int np = std::min(chunk, npairs - pair0);
    cesim_status st = CESIM_OK;
    if (draw_chunk_pow2<real>(t1, t2, buf, fields, m1, m2, np, tw1, tw2, slb, key, nreal, pair0,
                              shape, c->timer, s, st)) {
      CESIM_TRY(st);
      continue;
    }
    int tr = c->timer.begin(ST_DRAW_PASS_A, s);
    CESIM_TRY((launch_cols_noise<real>(buf, t1, t2, m2, np, c->tt.p2, tw2, sl, key, nreal, pair0,
                                       s)));
    c->timer.end(tr, s);
    tr = c->timer.begin(ST_DRAW_PASS_B, s);
    CESIM_TRY((launch_rows_crop<real>(buf, fields, t1, m1, m2, np, c->tt.p1, tw1, key, nreal,
                                      pair0, s)));
    c->timer.end(tr, s);
  }
  return CESIM_OK;
}

}  // namespace

bool register_draw_torus(int t1, int t2) {
  if (t1 != t2) return false;
  switch (t1) {
    case 128: case 256: case 512: case 1024: case 2048: case 4096: case 8192: return true;
    case 384: case 768: case 1536: case 3072: case 6144: return true;
    default: return false;
  }
}

bool register_draw_path(cesim_ctx c) { return register_draw_torus(c->t1, c->t2); }

DrawShape draw_shape_limits(cesim_ctx c) {
  const bool f64 = c->prec == CESIM_PREC_FP64;
  switch (c->t1) {
#define CESIM_LIM(TT) \
  case TT: return f64 ? clamp_shape<double, TT, TT>(DrawShape{}) : clamp_shape<float, TT, TT>(DrawShape{});
    CESIM_LIM(128) CESIM_LIM(256) CESIM_LIM(512) CESIM_LIM(1024) CESIM_LIM(2048) CESIM_LIM(4096)
    CESIM_LIM(8192)
    CESIM_LIM(384) CESIM_LIM(768) CESIM_LIM(1536) CESIM_LIM(3072) CESIM_LIM(6144)
#undef CESIM_LIM
    default: return DrawShape{0, 1};
  }
}

// Bytes of one pair's buffer between the passes: the m2 kept rows of the
// column transform, complex, in the path's precision.
size_t draw_pair_bytes(cesim_ctx c) {
  const size_t el = c->prec == CESIM_PREC_FP64 ? sizeof(double2) : sizeof(float2);
  return el * (size_t)c->t1 * c->grid.m2;
}

// Pairs a call of nreal realizations from first_real touches: absolute
// pairs floor(first / 2) .. floor((first + nreal - 1) / 2).  A context whose
// realization offset is read on the device (a captured batch, replayed at
// offsets of either parity) takes nreal / 2 + 1, one of which may be spare.
int draw_npairs(cesim_ctx c, int nreal, int first_real) {
  if (c->roff) return nreal / 2 + 1;
  return ((first_real + nreal - 1) >> 1) - (first_real >> 1) + 1;
}

// Pairs per draw launch: all of them within a 2 GiB buffer, or the count
// set with CESIM_PARAM_DRAW_CHUNK_PAIRS.
int draw_chunk_pairs(cesim_ctx c, int nreal, int first_real) {
  const int npairs = draw_npairs(c, nreal, first_real);
  const size_t budget = (size_t)2 << 30;
  int chunk = (int)std::max<size_t>(1, std::min<size_t>(npairs, budget / draw_pair_bytes(c)));
  if (c->draw_chunk_pairs > 0) chunk = std::min(npairs, c->draw_chunk_pairs);
  return chunk;
}

// d sqrt(lambda / N) / dtheta from dlambda = Re FFT2 of the theta-derivative
// of the base (in buf) and s = sqrt(lambda / N); zero where lambda <= 1e-12
// lambda_max, where the setup clamps lambda.
__global__ void k_dsqrt_lambda(const double2* __restrict__ dlam, const double* __restrict__ s,
                               size_t N, double lam_floor, double* __restrict__ ds) {
  const size_t q = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (q >= N) return;
  const double lam = s[q] * s[q] * (double)N;
  ds[q] = lam > lam_floor ? dlam[q].x / (2.0 * s[q] * (double)N) : 0.0;
}

__global__ void k_scale_complex(const double2* __restrict__ a, const double* __restrict__ m,
                                size_t N, double2* __restrict__ out) {
  const size_t q = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (q < N) out[q] = {a[q].x * m[q], a[q].y * m[q]};
}

__global__ void k_crop_real(const double2* __restrict__ a, int t1, int m1, int m2,
                            double* __restrict__ out) {
  const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (size_t)m1 * m2) return;
  const int j = (int)(e / m1), i = (int)(e % m1);
  out[e] = a[(size_t)j * t1 + i].x;
}

// ds = d sqrt(lambda / N) / dtheta ([T2][T1], FP64) from the FFT of the
// torus base's theta-derivative; tmp: N complex doubles of scratch.
cesim_status grad_dsqrt_device(cesim_ctx c, double* ds, double2* tmp) {
  hipStream_t s = c->stream;
  const int t1 = c->t1, t2 = c->t2;
  const size_t N = (size_t)t1 * t2;
  const unsigned nb = (unsigned)((N + 255) / 256);
  k_torus_base<true><<<dim3((t1 + 255) / 256, t2), 256, 0, s>>>(c->covd, c->grid.dx, c->grid.dy,
                                                                t1, t2, tmp);
  CESIM_HIP(hipGetLastError());
  CESIM_TRY(fft2_forward<double>(tmp, t1, t2, c->tt.p1, c->tt.p2, c->tt.tw1_64.as<double2>(),
                                 c->tt.tw2_64.as<double2>(), s));
  k_dsqrt_lambda<<<nb, 256, 0, s>>>(tmp, c->s64.as<double>(), N, 1e-12 * c->lam_max, ds);
  CESIM_HIP(hipGetLastError());
  return CESIM_OK;
}

// The FP64 draw of realizations first_real .. + nreal - 1 (on either
// context precision) with the spectrum sl ([T2][T1]) in place of
// sqrt(lambda / N): ds gives the fields' theta-derivatives.  slb: N doubles
// of scratch for the copy blocked by 8 columns that the register path reads.
cesim_status draw_f64_spectrum_device(cesim_ctx c, int nreal, uint64_t seed, int first_real,
                                      double* fields, const double* sl, double* slb) {
  const int t1 = c->t1, t2 = c->t2;
  const size_t N = (size_t)t1 * t2;
  const bool reg = register_draw_torus(t1, t2);
  if (reg) {
    k_block_lambda<double><<<(unsigned)((N + 255) / 256), 256, 0, c->stream>>>(sl, t1, t2, slb);
    CESIM_HIP(hipGetLastError());
  }
  return draw_typed<double>(c, nreal, seed, first_real, fields, c->tt.tw1_64.as<double2>(),
                            c->tt.tw2_64.as<double2>(), sl, reg ? slb : nullptr, nullptr, 0);
}

// Mean-noise fields of the linear-statistic gradient (FP64, general FFT
// passes on one buffer): with the complex mean noise zeta_bar,
// yb = crop(Re FFT2(s zeta_bar)) and dyb = crop(Re FFT2(ds zeta_bar)),
// [m2][m1], s = sqrt(lambda / N) and ds its theta-derivative.
cesim_status ce_grad_fields_device(cesim_ctx c, const double2* zeta_bar, double* yb, double* dyb) {
  hipStream_t s = c->stream;
  const int t1 = c->t1, t2 = c->t2, m1 = c->grid.m1, m2 = c->grid.m2;
  const size_t N = (size_t)t1 * t2;
  CESIM_TRY(c->gwork.reserve(sizeof(double2) * N + sizeof(double) * N));
  double2* buf = c->gwork.as<double2>();
  double* ds = reinterpret_cast<double*>(buf + N);
  const double2* tw1 = c->tt.tw1_64.as<double2>();
  const double2* tw2 = c->tt.tw2_64.as<double2>();
  const unsigned nb = (unsigned)((N + 255) / 256);
  CESIM_TRY(grad_dsqrt_device(c, ds, buf));
  const unsigned nm = (unsigned)(((size_t)m1 * m2 + 255) / 256);
  for (int pass = 0; pass < 2; ++pass) {
    k_scale_complex<<<nb, 256, 0, s>>>(zeta_bar, pass == 0 ? c->s64.as<double>() : ds, N, buf);
    CESIM_HIP(hipGetLastError());
    CESIM_TRY(fft2_forward<double>(buf, t1, t2, c->tt.p1, c->tt.p2, tw1, tw2, s));
    k_crop_real<<<nm, 256, 0, s>>>(buf, t1, m1, m2, pass == 0 ? yb : dyb);
    CESIM_HIP(hipGetLastError());
  }
  return CESIM_OK;
}

// ------------------------------------------- pair buffers without allocation
// The pair buffers of ce_simulate_noalloc: one array per device that runs
// the library, held until the process ends and shared by every such call on
// that device.  Host code never uses the array's name as an address: the
// device address comes from hipGetSymbolAddress, looked up once per device
// with that device current (ce_setup) and cached.
static __device__ __align__(256) unsigned char scratch[kDrawScratchBytes];

cesim_status draw_scratch_address(void** out) {
  static std::mutex mu;
  static std::vector<void*> addr;             // per device ordinal
  int dev = 0;
  CESIM_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(mu);
  if ((int)addr.size() <= dev) addr.resize(dev + 1, nullptr);
  if (!addr[dev]) {
    void* p = nullptr;
    CESIM_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    addr[dev] = p;
  }
  *out = addr[dev];
  return CESIM_OK;
}

cesim_status ce_draw_device(cesim_ctx c, int nreal, uint64_t seed, int first_real, void* fields,
                            void* work, size_t work_bytes) {
  if (c->ext_work && !work) {       // pair buffers lent by a batch
    work = c->ext_work;
    work_bytes = c->ext_work_bytes;
  }
  if (c->prec == CESIM_PREC_FP64)
    return draw_typed<double>(c, nreal, seed, first_real, static_cast<double*>(fields),
                              c->tt.tw1_64.as<double2>(), c->tt.tw2_64.as<double2>(),
                              c->s64.as<double>(), c->slb.as<double>(), work, work_bytes);
  return draw_typed<float>(c, nreal, seed, first_real, static_cast<float*>(fields),
                           c->tt.tw1_32.as<float2>(), c->tt.tw2_32.as<float2>(),
                           c->s32.as<float>(), c->slb.as<float>(), work, work_bytes);
}

}  // namespace cesim
