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

// Noise for torus rows [j0, j0 + nrows) of pair p into LDS as
// eps_{r0} + i eps_{r1}; element q = j t1 + i uses block q / 4, word q % 4.
template <typename real, int NTHR>
__device__ void noise_rows(cpx<real>* lds, int t1, int j0, int nrows, const NoiseKey& key,
                           int r0, bool has_r1) {
  const uint32_t k0 = key.k0, k1 = key.k1, ev = key.event;
  const long q_lo = (long)j0 * t1;
  const long q_hi = q_lo + (long)nrows * t1;
  const long b_lo = q_lo >> 2, b_hi = (q_hi - 1) >> 2;
  for (long b = b_lo + threadIdx.x; b <= b_hi; b += NTHR) {
    real za[4], zb[4] = {0, 0, 0, 0};
    if constexpr (sizeof(real) == 8) {
      normals4_f64(k0, k1, (uint32_t)b, (uint32_t)r0, ev, 0u, za);
      if (has_r1) normals4_f64(k0, k1, (uint32_t)b, (uint32_t)(r0 + 1), ev, 0u, zb);
    } else {
      normals4_f32(k0, k1, (uint32_t)b, (uint32_t)r0, ev, 0u, za);
      if (has_r1) normals4_f32(k0, k1, (uint32_t)b, (uint32_t)(r0 + 1), ev, 0u, zb);
    }
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      const long q = 4 * b + w;
      if (q >= q_lo && q < q_hi) lds[q - q_lo] = {za[w], zb[w]};
    }
  }
}

// Forward FFT of nb torus rows per workgroup.  NOISE: the input is the pair
// noise; otherwise it is read from buf.  Output overwrites buf.
template <typename real, int NTHR, int E, bool NOISE>
__global__ void __launch_bounds__(NTHR)
k_rows_fwd(cpx<real>* __restrict__ buf, int t1, int t2, int nb, Plan plan,
           const cpx<real>* __restrict__ tw, bool tw_lds, NoiseKey key, int nreal, int pair0) {
  extern __shared__ __align__(16) unsigned char smem[];
  cpx<real>* lds = reinterpret_cast<cpx<real>*>(smem);
  const int p = blockIdx.y;
  const int j0 = blockIdx.x * nb;
  const int nr = min(nb, t2 - j0);
  cpx<real>* base = buf + ((size_t)p * t2 + j0) * t1;
  const cpx<real>* twl = stage_twiddles<real, NTHR>(lds + nb * t1, tw, t1, tw_lds);
  if constexpr (NOISE) {
    const int pg = pair0 + p;               // pair index within this call
    const int r0 = key.base() + 2 * pg;
    noise_rows<real, NTHR>(lds, t1, j0, nr, key, r0, 2 * pg + 1 < nreal);
  } else {
    for (int e = threadIdx.x; e < nr * t1; e += NTHR) lds[e] = base[e];
  }
  __syncthreads();
  fft_lds<false, NTHR, E, false, real>(lds, plan, nr, 1, t1, twl);
  for (int e = threadIdx.x; e < nr * t1; e += NTHR) base[e] = lds[e];
}

// Column panel of cp columns of every pair: forward FFT along y; with SCALE
// also multiply by s[ky][kx] and inverse FFT along y, writing rows < rows_out.
template <typename real, int NTHR, int E, bool SCALE>
__global__ void __launch_bounds__(NTHR)
k_cols(cpx<real>* __restrict__ buf, int t1, int t2, int cp, int rows_out, Plan plan,
       const cpx<real>* __restrict__ tw, bool tw_lds, const real* __restrict__ s) {
  extern __shared__ __align__(16) unsigned char smem[];
  cpx<real>* lds = reinterpret_cast<cpx<real>*>(smem);
  const cpx<real>* twl = stage_twiddles<real, NTHR>(lds + cp * t2, tw, t2, tw_lds);
  const int p = blockIdx.y;
  const int c0 = blockIdx.x * cp;
  const int cw = min(cp, t1 - c0);
  cpx<real>* base = buf + (size_t)p * t2 * t1 + c0;
  for (int e = threadIdx.x; e < t2 * cp; e += NTHR) {
    const int row = e / cp, c = e - row * cp;
    lds[e] = c < cw ? base[(size_t)row * t1 + c] : cpx<real>{0, 0};
  }
  __syncthreads();
  fft_lds<false, NTHR, E, true, real>(lds, plan, cp, cp, 1, twl);
  if constexpr (SCALE) {
    for (int e = threadIdx.x; e < t2 * cp; e += NTHR) {
      const int row = e / cp, c = e - row * cp;
      if (c < cw) {
        const real m = s[(size_t)row * t1 + c0 + c];
        lds[e] = {lds[e].x * m, lds[e].y * m};
      }
    }
    __syncthreads();
    fft_lds<true, NTHR, E, true, real>(lds, plan, cp, cp, 1, twl);
  }
  for (int e = threadIdx.x; e < rows_out * cp; e += NTHR) {
    const int row = e / cp, c = e - row * cp;
    if (c < cw) base[(size_t)row * t1 + c] = lds[e];
  }
}

// Inverse FFT along x of nb kept rows (y < m2) and the crop: the first m1
// outputs of the row of pair p become fields 2p (real) and 2p+1 (imag).
template <typename real, int NTHR, int E>
__global__ void __launch_bounds__(NTHR)
k_rows_inv_crop(const cpx<real>* __restrict__ buf, real* __restrict__ fields, int t1, int t2,
                int m1, int m2, int nb, Plan plan, const cpx<real>* __restrict__ tw, bool tw_lds,
                int nreal, int pair0) {
  extern __shared__ __align__(16) unsigned char smem[];
  cpx<real>* lds = reinterpret_cast<cpx<real>*>(smem);
  const cpx<real>* twl = stage_twiddles<real, NTHR>(lds + nb * t1, tw, t1, tw_lds);
  const int p = blockIdx.y;
  const int j0 = blockIdx.x * nb;
  const int nr = min(nb, m2 - j0);
  const cpx<real>* base = buf + ((size_t)p * t2 + j0) * t1;
  for (int e = threadIdx.x; e < nr * t1; e += NTHR) lds[e] = base[e];
  __syncthreads();
  fft_lds<true, NTHR, E, false, real>(lds, plan, nr, 1, t1, twl);
  const int pg = pair0 + p;
  const size_t M = (size_t)m1 * m2;
  real* f0 = fields + (size_t)(2 * pg) * M + (size_t)j0 * m1;
  const bool has1 = 2 * pg + 1 < nreal;
  for (int e = threadIdx.x; e < nr * m1; e += NTHR) {
    const int row = e / m1, x = e - row * m1;
    const cpx<real> v = lds[row * t1 + x];
    f0[(size_t)row * m1 + x] = v.x;
    if (has1) f0[M + (size_t)row * m1 + x] = v.y;
  }
}

// ------------------------------------------- power-of-two draw kernels
// Same three passes as above with the transform length fixed at compile
// time and the data held in registers (see fft_pow2.hpp).

// Pass 1: noise of ROWS torus rows (natural order into LDS), forward row
// FFT, result written from registers.
template <typename real, int T>
__global__ void __launch_bounds__(P2Rows<T>::NTHR)
k_p2_rows_noise(cpx<real>* __restrict__ buf, int t2, const cpx<real>* __restrict__ tw, NoiseKey key,
                int nreal, int pair0) {
  using C = cpx<real>;
  using G = P2Rows<T>;
  extern __shared__ __align__(16) unsigned char smem[];
  C* lds = reinterpret_cast<C*>(smem);
  const int p = blockIdx.y;
  const int rows = blockDim.x / G::S;
  const int j0 = blockIdx.x * rows;
  const int pg = pair0 + p;
  const int r0 = key.base() + 2 * pg;
  const bool has1 = 2 * pg + 1 < nreal;
  const uint32_t k0 = key.k0, k1 = key.k1, ev = key.event;
  // Philox blocks of 4 consecutive elements; T is a multiple of 4, so a
  // block never straddles two rows.
  constexpr int BPR = T / 4;
  for (int blk = threadIdx.x; blk < rows * BPR; blk += blockDim.x) {
    const int b = blk / BPR, i0 = (blk % BPR) * 4;
    if (j0 + b >= t2) continue;
    const uint32_t gb = (uint32_t)((((long)(j0 + b)) * T + i0) >> 2);
    real za[4], zb[4] = {0, 0, 0, 0};
    if constexpr (sizeof(real) == 8) {
      normals4_f64(k0, k1, gb, (uint32_t)r0, ev, 0u, za);
      if (has1) normals4_f64(k0, k1, gb, (uint32_t)(r0 + 1), ev, 0u, zb);
    } else {
      normals4_f32(k0, k1, gb, (uint32_t)r0, ev, 0u, za);
      if (has1) normals4_f32(k0, k1, gb, (uint32_t)(r0 + 1), ev, 0u, zb);
    }
    const RowLds<C> rl{lds + b * G::LD};
#pragma unroll
    for (int w = 0; w < 4; ++w) rl.store(i0 + w, C{za[w], zb[w]});
  }
  __syncthreads();
  const int b = threadIdx.x / G::S, base = threadIdx.x % G::S;
  const RowLds<C> rl{lds + b * G::LD};
  C x[G::E];
#pragma unroll
  for (int h = 0; h < G::E; ++h) x[h] = rl.load(base + G::S * h);
  p2_fft<real, T, false>(x, base, tw, rl);
  if (j0 + b < t2) {
    C* out = buf + ((size_t)p * t2 + j0 + b) * T;
#pragma unroll
    for (int h = 0; h < G::E; ++h) out[base + G::S * h] = x[h];
  }
}

// Pass 2: CP columns per workgroup, loaded straight into registers; forward
// FFT along y, sqrt(lambda)/N in registers (from the copy blocked by 8
// columns, so that a wave reads 8 rows of 8 columns contiguously), inverse
// FFT, rows < rows_out stored.
template <typename real, int T>
__global__ void __launch_bounds__((P2Cols<real, T>::NTHR))
k_p2_cols(cpx<real>* __restrict__ buf, int t1, int rows_out, const cpx<real>* __restrict__ tw,
          const real* __restrict__ slb, int lcp) {
  using C = cpx<real>;
  using G = P2Cols<real, T>;
  extern __shared__ __align__(16) unsigned char smem[];
  C* lds = reinterpret_cast<C*>(smem);
  const int p = blockIdx.y;
  const int cp = 1 << lcp;
  const int c = threadIdx.x & (cp - 1), base = threadIdx.x >> lcp;
  // Workgroups are dealt to the 8 XCDs round-robin; when the panel count is
  // a multiple of 8, panels are renumbered so that one XCD takes adjacent
  // panels in turn and the halves of each cache line meet in its L2.
  int panel = blockIdx.x;
  if ((gridDim.x & 7) == 0) panel = (blockIdx.x & 7) * (gridDim.x >> 3) + (blockIdx.x >> 3);
  const int col = panel * cp + c;
  const bool ok = col < t1;
  C* colp = buf + (size_t)p * T * t1 + col;
  C x[G::E];
#pragma unroll
  for (int h = 0; h < G::E; ++h) x[h] = ok ? colp[(size_t)(base + G::S * h) * t1] : C{0, 0};
  const ColLds<C> cl{lds, c, lcp};
  p2_fft<real, T, false>(x, base, tw, cl);
#pragma unroll
  for (int h = 0; h < G::E; ++h) {
    const real m = ok ? slb[((size_t)(col >> 3) * T + base + G::S * h) * 8 + (col & 7)] : (real)0;
    x[h] = {x[h].x * m, x[h].y * m};
  }
  p2_fft<real, T, true>(x, base, tw, cl);
  if (ok) {
#pragma unroll
    for (int h = 0; h < G::E; ++h) {
      const int row = base + G::S * h;
      if (row < rows_out) colp[(size_t)row * t1] = x[h];
    }
  }
}

// Pass 3: ROWS kept rows per workgroup: inverse row FFT and the crop into
// fields 2p (real part) and 2p+1 (imaginary part).
template <typename real, int T>
__global__ void __launch_bounds__(P2Rows<T>::NTHR)
k_p2_rows_inv_crop(const cpx<real>* __restrict__ buf, real* __restrict__ fields, int t2, int m1,
                   int m2, const cpx<real>* __restrict__ tw, int nreal, int pair0) {
  using C = cpx<real>;
  using G = P2Rows<T>;
  extern __shared__ __align__(16) unsigned char smem[];
  C* lds = reinterpret_cast<C*>(smem);
  const int p = blockIdx.y;
  const int b = threadIdx.x / G::S, base = threadIdx.x % G::S;
  const int j = blockIdx.x * (blockDim.x / G::S) + b;
  const bool ok = j < m2;
  const C* in = buf + ((size_t)p * t2 + (ok ? j : 0)) * T;
  C x[G::E];
#pragma unroll
  for (int h = 0; h < G::E; ++h) x[h] = ok ? in[base + G::S * h] : C{0, 0};
  const RowLds<C> rl{lds + b * G::LD};
  p2_fft<real, T, true>(x, base, tw, rl);
  if (!ok) return;
  const int pg = pair0 + p;
  const size_t M = (size_t)m1 * m2;
  real* f0 = fields + (size_t)(2 * pg) * M + (size_t)j * m1;
  const bool has1 = 2 * pg + 1 < nreal;
#pragma unroll
  for (int h = 0; h < G::E; ++h) {
    const int xcol = base + G::S * h;
    if (xcol < m1) {
      f0[xcol] = x[h].x;
      if (has1) f0[M + xcol] = x[h].y;
    }
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

__global__ void k_sqrt_lambda(const double2* lam, size_t N, double inv_n, double* s64, float* s32) {
  const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= N) return;
  const double v = sqrt(fmax(lam[q].x, 0.0)) * inv_n;
  s64[q] = v;
  if (s32) s32[q] = (float)v;
}

// sqrt(lambda) / N of the register draw path, in the path's precision and
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

template <typename real, bool NOISE>
cesim_status launch_rows_fwd(cpx<real>* buf, int t1, int t2, int npairs, const Plan& plan,
                             const cpx<real>* tw, const NoiseKey& key, int nreal, int pair0,
                             hipStream_t s) {
  int nb, E;
  bool twl;
  size_t lds;
  row_config<real>(t1, nb, E, twl, lds);
  dim3 grid((t2 + nb - 1) / nb, npairs);
  if (E == 16) {
    auto k = k_rows_fwd<real, kRowThreads, 16, NOISE>;
    allow_lds(k, lds);
    k<<<grid, kRowThreads, lds, s>>>(buf, t1, t2, nb, plan, tw, twl, key, nreal, pair0);
  } else {
    auto k = k_rows_fwd<real, kRowThreads, 32, NOISE>;
    allow_lds(k, lds);
    k<<<grid, kRowThreads, lds, s>>>(buf, t1, t2, nb, plan, tw, twl, key, nreal, pair0);
  }
  CESIM_HIP(hipGetLastError());
  return CESIM_OK;
}

template <typename real, bool SCALE>
cesim_status launch_cols(cpx<real>* buf, int t1, int t2, int npairs, int rows_out, const Plan& plan,
                         const cpx<real>* tw, const real* sl, hipStream_t s) {
  int cp, E;
  bool twl;
  size_t lds;
  col_config<real>(t2, t1, cp, E, twl, lds);
  dim3 grid((t1 + cp - 1) / cp, npairs);
#define CESIM_COLS(EE)                                                            \
  {                                                                               \
    auto k = k_cols<real, kColThreads, EE, SCALE>;                                \
    allow_lds(k, lds);                                                            \
    k<<<grid, kColThreads, lds, s>>>(buf, t1, t2, cp, rows_out, plan, tw, twl, sl); \
  }
  switch (E) {
    case 4: CESIM_COLS(4) break;
    case 8: CESIM_COLS(8) break;
    case 16: CESIM_COLS(16) break;
    default: CESIM_COLS(32) break;
  }
#undef CESIM_COLS
  CESIM_HIP(hipGetLastError());
  return CESIM_OK;
}

template <typename real>
cesim_status launch_rows_inv_crop(const cpx<real>* buf, real* fields, int t1, int t2, int m1,
                                  int m2, int npairs, const Plan& plan, const cpx<real>* tw,
                                  int nreal, int pair0, hipStream_t s) {
  int nb, E;
  bool twl;
  size_t lds;
  row_config<real>(t1, nb, E, twl, lds);
  dim3 grid((m2 + nb - 1) / nb, npairs);
  if (E == 16) {
    auto k = k_rows_inv_crop<real, kRowThreads, 16>;
    allow_lds(k, lds);
    k<<<grid, kRowThreads, lds, s>>>(buf, fields, t1, t2, m1, m2, nb, plan, tw, twl, nreal,
                                     pair0);
  } else {
    auto k = k_rows_inv_crop<real, kRowThreads, 32>;
    allow_lds(k, lds);
    k<<<grid, kRowThreads, lds, s>>>(buf, fields, t1, t2, m1, m2, nb, plan, tw, twl, nreal,
                                     pair0);
  }
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
  CESIM_TRY((launch_rows_fwd<double, false>(buf, t1, t2, 1, p1, c->tt.tw1_64.as<double2>(),
                                            NoiseKey{}, 0, 0, s)));
  CESIM_TRY((launch_cols<double, false>(buf, t1, t2, 1, t2, p2, c->tt.tw2_64.as<double2>(),
                                        nullptr, s)));
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
  k_sqrt_lambda<<<(unsigned)((N + 255) / 256), 256, 0, s>>>(buf, N, 1.0 / (double)N,
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

// Tile shape of the register path: rows per workgroup of passes 1 and 3 and
// log2 of the columns per workgroup of pass 2, clamped to each kernel's
// maximum (results do not depend on it).
template <typename real, int T1, int T2>
DrawShape clamp_shape(DrawShape d) {
  using GR = P2Rows<T1>;
  using GC = P2Cols<real, T2>;
  auto fix_rows = [](int r) {
    int v = GR::ROWS;
    if (r > 0) while (v > 1 && v > r) v >>= 1;
    return v;
  };
  d.rows1 = fix_rows(d.rows1);
  d.rows3 = fix_rows(d.rows3);
  const int lmax = ilog2c(GC::CP);
  d.lcp2 = (d.lcp2 < 0 || d.lcp2 > lmax) ? lmax : d.lcp2;
  return d;
}

template <typename real, int T1, int T2>
cesim_status draw_chunk_p2(cpx<real>* buf, real* fields, int m1, int m2, int np, const cpx<real>* tw1,
                           const cpx<real>* tw2, const real* slb, const NoiseKey& key, int nreal,
                           int pair0, const DrawShape& shape, StageTimer& tm, hipStream_t s) {
  using GR = P2Rows<T1>;
  using GC = P2Cols<real, T2>;
  const DrawShape d = clamp_shape<real, T1, T2>(shape);
  const int cp = 1 << d.lcp2;
  const size_t lr1 = sizeof(cpx<real>) * d.rows1 * GR::LD;
  const size_t lr3 = sizeof(cpx<real>) * d.rows3 * GR::LD;
  const size_t lc = sizeof(cpx<real>) * cp * GC::LD;
  int tr = tm.begin(ST_DRAW_PASS1, s);
  {
    auto k = k_p2_rows_noise<real, T1>;
    allow_lds(k, sizeof(cpx<real>) * GR::ROWS * GR::LD);
    k<<<dim3((T2 + d.rows1 - 1) / d.rows1, np), d.rows1 * GR::S, lr1, s>>>(buf, T2, tw1, key,
                                                                           nreal, pair0);
    CESIM_HIP(hipGetLastError());
  }
  tm.end(tr, s);
  tr = tm.begin(ST_DRAW_PASS2, s);
  {
    auto k = k_p2_cols<real, T2>;
    allow_lds(k, sizeof(cpx<real>) * GC::CP * GC::LD);
    k<<<dim3((T1 + cp - 1) / cp, np), cp * GC::S, lc, s>>>(buf, T1, m2, tw2, slb, d.lcp2);
    CESIM_HIP(hipGetLastError());
  }
  tm.end(tr, s);
  tr = tm.begin(ST_DRAW_PASS3, s);
  {
    auto k = k_p2_rows_inv_crop<real, T1>;
    allow_lds(k, sizeof(cpx<real>) * GR::ROWS * GR::LD);
    k<<<dim3((m2 + d.rows3 - 1) / d.rows3, np), d.rows3 * GR::S, lr3, s>>>(buf, fields, T2, m1,
                                                                           m2, tw1, nreal, pair0);
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
                        const real* slb) {
  hipStream_t s = c->stream;
  const int t1 = c->t1, t2 = c->t2, m1 = c->grid.m1, m2 = c->grid.m2;
  const size_t pair_bytes = sizeof(cpx<real>) * (size_t)t1 * t2;
  const int npairs = (nreal + 1) / 2;
  int chunk = draw_chunk_pairs(c, nreal);
  cpx<real>* buf;
  if (c->ext_work) {                // pair buffers lent by a batch
    chunk = std::min<size_t>(chunk, c->ext_work_bytes / pair_bytes);
    if (chunk < 1) return CESIM_ERR_INVALID_ARG;
    buf = static_cast<cpx<real>*>(c->ext_work);
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
    int tr = c->timer.begin(ST_DRAW_PASS1, s);
    CESIM_TRY((launch_rows_fwd<real, true>(buf, t1, t2, np, c->tt.p1, tw1, key, nreal, pair0, s)));
    c->timer.end(tr, s);
    tr = c->timer.begin(ST_DRAW_PASS2, s);
    CESIM_TRY((launch_cols<real, true>(buf, t1, t2, np, m2, c->tt.p2, tw2, sl, s)));
    c->timer.end(tr, s);
    tr = c->timer.begin(ST_DRAW_PASS3, s);
    CESIM_TRY((launch_rows_inv_crop<real>(buf, fields, t1, t2, m1, m2, np, c->tt.p1, tw1, nreal,
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
    default: return DrawShape{1, 0, 1};
  }
}

size_t draw_pair_bytes(cesim_ctx c) {
  const size_t el = c->prec == CESIM_PREC_FP64 ? sizeof(double2) : sizeof(float2);
  return el * (size_t)c->t1 * c->t2;
}

// Pairs per draw launch: all of them within a 2 GiB buffer, or the count
// set with CESIM_PARAM_DRAW_CHUNK_PAIRS.
int draw_chunk_pairs(cesim_ctx c, int nreal) {
  const int npairs = (nreal + 1) / 2;
  const size_t budget = (size_t)2 << 30;
  int chunk = (int)std::max<size_t>(1, std::min<size_t>(npairs, budget / draw_pair_bytes(c)));
  if (c->draw_chunk_pairs > 0) chunk = std::min(npairs, c->draw_chunk_pairs);
  return chunk;
}

// d sqrt(lambda)/dtheta / N from dlambda = Re FFT2 of the theta-derivative of
// the base (in buf) and s = sqrt(lambda) / N; zero where lambda <= 1e-12
// lambda_max, where the setup clamps lambda.
__global__ void k_dsqrt_lambda(const double2* __restrict__ dlam, const double* __restrict__ s,
                               size_t N, double lam_floor, double* __restrict__ ds) {
  const size_t q = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (q >= N) return;
  const double sq = s[q] * (double)N;          // sqrt(lambda)
  ds[q] = (sq * sq > lam_floor) ? dlam[q].x / (2.0 * sq * (double)N) : 0.0;
}

__global__ void k_real_to_complex(const double* __restrict__ a, size_t N, double2* __restrict__ out) {
  const size_t q = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (q < N) out[q] = {a[q], 0.0};
}

// Mean-noise fields of the linear-statistic gradient (FP64, general FFT
// passes on one pair buffer): yb = crop(F^-1 diag(sqrt(lambda)) F eps_bar)
// and dyb = crop(F^-1 diag(d sqrt(lambda)/dtheta) F eps_bar), [m2][m1].
cesim_status ce_grad_fields_device(cesim_ctx c, const double* eps_bar, double* yb, double* dyb) {
  hipStream_t s = c->stream;
  const int t1 = c->t1, t2 = c->t2, m1 = c->grid.m1, m2 = c->grid.m2;
  const size_t N = (size_t)t1 * t2;
  CESIM_TRY(c->gwork.reserve(sizeof(double2) * N + sizeof(double) * N));
  double2* buf = c->gwork.as<double2>();
  double* ds = reinterpret_cast<double*>(buf + N);
  const double2* tw1 = c->tt.tw1_64.as<double2>();
  const double2* tw2 = c->tt.tw2_64.as<double2>();
  const unsigned nb = (unsigned)((N + 255) / 256);
  k_torus_base<true><<<dim3((t1 + 255) / 256, t2), 256, 0, s>>>(c->covd, c->grid.dx, c->grid.dy,
                                                                t1, t2, buf);
  CESIM_HIP(hipGetLastError());
  CESIM_TRY((launch_rows_fwd<double, false>(buf, t1, t2, 1, c->tt.p1, tw1, NoiseKey{}, 0, 0, s)));
  CESIM_TRY((launch_cols<double, false>(buf, t1, t2, 1, t2, c->tt.p2, tw2, nullptr, s)));
  k_dsqrt_lambda<<<nb, 256, 0, s>>>(buf, c->s64.as<double>(), N, 1e-12 * c->lam_max, ds);
  CESIM_HIP(hipGetLastError());
  for (int pass = 0; pass < 2; ++pass) {
    k_real_to_complex<<<nb, 256, 0, s>>>(eps_bar, N, buf);
    CESIM_HIP(hipGetLastError());
    CESIM_TRY((launch_rows_fwd<double, false>(buf, t1, t2, 1, c->tt.p1, tw1, NoiseKey{}, 0, 0, s)));
    CESIM_TRY((launch_cols<double, true>(buf, t1, t2, 1, m2, c->tt.p2, tw2,
                                         pass == 0 ? c->s64.as<double>() : ds, s)));
    CESIM_TRY((launch_rows_inv_crop<double>(buf, pass == 0 ? yb : dyb, t1, t2, m1, m2, 1,
                                            c->tt.p1, tw1, 1, 0, s)));
  }
  return CESIM_OK;
}

cesim_status ce_draw_device(cesim_ctx c, int nreal, uint64_t seed, int first_real, void* fields) {
  if (c->prec == CESIM_PREC_FP64)
    return draw_typed<double>(c, nreal, seed, first_real, static_cast<double*>(fields),
                              c->tt.tw1_64.as<double2>(), c->tt.tw2_64.as<double2>(),
                              c->s64.as<double>(), c->slb.as<double>());
  return draw_typed<float>(c, nreal, seed, first_real, static_cast<float*>(fields),
                           c->tt.tw1_32.as<float2>(), c->tt.tw2_32.as<float2>(),
                           c->s32.as<float>(), c->slb.as<float>());
}

}  // namespace cesim
