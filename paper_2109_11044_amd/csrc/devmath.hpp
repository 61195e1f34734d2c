// devmath.hpp -- covariance model, Philox4x32-10 and Box-Muller for the
// gfx950 kernels.  FP64 routines are __host__ __device__ so that the host
// test hooks of the C ABI evaluate exactly this source.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <math.h>

namespace cesim {

// ---------------------------------------------------------------- constants
constexpr double kEuler = 0.57721566490153286061;   // Euler-Mascheroni
constexpr double kSqrt2 = 1.4142135623730950488;
constexpr double kSqrt3 = 1.7320508075688772935;
constexpr double kLog2e = 1.4426950408889634074;
constexpr double kSqrtHalfPi = 1.2533141373155002512;   // sqrt(pi / 2)

// cosh(j / 8), j = 0..31: abscissae of the trapezoidal rule for K_1 below.
#define CESIM_COSH_EIGHTHS                                                    \
  1.0, 1.0078226778257108598, 1.0314130998795731762, 1.0711403467045867673,   \
  1.1276259652063807852, 1.2017536929756063242, 1.2946832846768446878,        \
  1.4078686568228031586, 1.5430806348152437785, 1.7024346581381904874,        \
  1.8884238771610157382, 2.103958159362661802, 2.3524096152432473258,         \
  2.6376653561921375823, 2.9641883097280877818, 3.3370870435875205143,        \
  3.7621956910836314596, 4.2461652281969921406, 4.7965675304601950287,        \
  5.4220138376435092506, 6.1322894796636861166, 6.938506971550673191,         \
  7.8532798726974395915, 8.8909201304827093218, 10.067661995777765842,        \
  11.4019160135750677, 12.914557062512392049, 14.629250949773302935,          \
  16.572824671057316126, 18.7756861284686772, 21.272299872959396082,          \
  24.101726314486257781

constexpr double kCoshEighths[32] = {CESIM_COSH_EIGHTHS};

__host__ __device__ inline double cosh_eighth(int j) { return kCoshEighths[j]; }

// ---------------------------------------------------------- covariance model
// Matern covariance of Section 3.3 for nu in {1/2, 1, 3/2}.  The anisotropic
// lag length in range units, x = d / theta, is |U h| for the 2x2 map
// U = diag(1, a) R(-phi) / theta, i.e. (u, a w) / theta with (u, w) the lag
// rotated into the major-axis frame.
struct CovDev {
  int nu_code;        // 0: nu = 1/2, 1: nu = 1, 2: nu = 3/2
  double sigma2;
  double u00, u01, u10, u11;
  double theta;       // range (U is proportional to 1 / theta)
};

// t K_1(t) for t >= 0 (equals 1 at t = 0), FP64.
//  t <= 2: ascending series (Abramowitz and Stegun 9.6.11 with n = 1):
//    t K_1(t) = 1 + t ln(t/2) I_1(t)
//               - (t^2/4) sum_k [psi(k+1) + psi(k+2)] (t^2/4)^k / (k!(k+1)!),
//    t I_1(t) = (t^2/2) sum_k (t^2/4)^k / (k!(k+1)!).
//  2 < t <= 30: trapezoidal rule with step 1/8 on the integral
//    representation K_1(t) = int_0^inf exp(-t cosh u) cosh u du, which
//    converges exponentially for this analytic, doubly-exponentially
//    decaying integrand (error ~ exp(t - 2 pi (pi/2) / h) < 1e-18 here);
//    32 nodes reach u = 3.875 where the integrand is below exp(-40) of its
//    peak for t > 2.
//  t > 30: Hankel's asymptotic expansion (A&S 9.7.2),
//    K_1(t) = sqrt(pi / (2t)) e^-t sum_k a_k, a_k = a_{k-1} (4 - (2k-1)^2) / (8 k t),
//    whose terms fall below 1e-17 within 22 terms for t > 30.
__host__ __device__ inline double t_bessel_k1(double t) {
  if (t <= 0.0) return 1.0;
  if (t <= 2.0) {
    const double q = 0.25 * t * t;
    double f = 1.0, si = 0.0, sp = 0.0;
    double psi1 = -kEuler;                         // psi(1)
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const double psi2 = psi1 + 1.0 / (double)(k + 1);   // psi(k+2)
      si += f;
      sp += (psi1 + psi2) * f;
      f *= q / (double)((k + 1) * (k + 2));
      psi1 = psi2;
    }
    return 1.0 + 2.0 * q * log(0.5 * t) * si - q * sp;
  }
  if (t <= 30.0) {
    double s = 0.5;                                // u = 0 node, halved
#pragma unroll 4
    for (int j = 1; j < 32; ++j) {
      const double c = cosh_eighth(j);
      s += exp(-t * (c - 1.0)) * c;
    }
    return t * exp(-t) * 0.125 * s;
  }
  double a = 1.0, s = 1.0;
#pragma unroll
  for (int k = 1; k < 22; ++k) {
    const double m = (double)(2 * k - 1);
    a *= (4.0 - m * m) / (8.0 * (double)k * t);
    s += a;
  }
  return kSqrtHalfPi * sqrt(t) * exp(-t) * s;
}

// Correlation rho_nu(x), x = d / theta >= 0, FP64.
__host__ __device__ inline double matern_rho(int nu_code, double x) {
  if (nu_code == 0) return exp(-x);
  if (nu_code == 2) {
    const double t = kSqrt3 * x;
    return (1.0 + t) * exp(-t);
  }
  return t_bessel_k1(kSqrt2 * x);
}

// t^2 K_0(t) for t >= 0 (0 at t = 0), FP64, in the three regimes of t K_1:
//  t <= 2: ascending series (Abramowitz and Stegun 9.6.13),
//    K_0(t) = -(ln(t/2) + gamma) I_0(t) + sum_{k>=1} H_k (t^2/4)^k / (k!)^2,
//    I_0(t) = sum_k (t^2/4)^k / (k!)^2,  H_k = 1 + 1/2 + ... + 1/k;
//  2 < t <= 30: the same trapezoidal rule on K_0(t) = int_0^inf exp(-t cosh u) du;
//  t > 30: Hankel's expansion (A&S 9.7.2) with 4 nu^2 = 0.
__host__ __device__ inline double t2_bessel_k0(double t) {
  if (t <= 0.0) return 0.0;
  if (t <= 2.0) {
    const double q = 0.25 * t * t;
    double f = 1.0, i0 = 0.0, sh = 0.0, h = 0.0;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      i0 += f;
      sh += h * f;                                 // H_k (t^2/4)^k / (k!)^2
      f *= q / (double)((k + 1) * (k + 1));
      h += 1.0 / (double)(k + 1);
    }
    return t * t * (sh - (log(0.5 * t) + kEuler) * i0);
  }
  if (t <= 30.0) {
    double s = 0.5;
#pragma unroll 4
    for (int j = 1; j < 32; ++j) s += exp(-t * (cosh_eighth(j) - 1.0));
    return t * t * exp(-t) * 0.125 * s;
  }
  double a = 1.0, s = 1.0;
#pragma unroll
  for (int k = 1; k < 22; ++k) {
    const double m = (double)(2 * k - 1);
    a *= -(m * m) / (8.0 * (double)k * t);
    s += a;
  }
  return kSqrtHalfPi * t * sqrt(t) * exp(-t) * s;
}

// g(x) = -x rho_nu'(x), x = d / theta, so that dC/dtheta = sigma^2 g(x) / theta:
// x e^-x (nu = 1/2), t^2 K_0(t) with t = sqrt(2) x (nu = 1, from
// d/dt [t K_1(t)] = -t K_0(t), A&S 9.6.28), t^2 e^-t with t = sqrt(3) x (nu = 3/2).
__host__ __device__ inline double matern_g(int nu_code, double x) {
  if (nu_code == 0) return x * exp(-x);
  if (nu_code == 2) {
    const double t = kSqrt3 * x;
    return t * t * exp(-t);
  }
  return t2_bessel_k0(kSqrt2 * x);
}

__host__ __device__ inline double lag_x(const CovDev& c, double hx, double hy) {
  const double a = c.u00 * hx + c.u01 * hy;
  const double b = c.u10 * hx + c.u11 * hy;
  return sqrt(a * a + b * b);
}

__host__ __device__ inline double cov_eval(const CovDev& c, double hx, double hy) {
  return c.sigma2 * matern_rho(c.nu_code, lag_x(c, hx, hy));
}

// dC(h) / dtheta (theta the range; the lag length in range units scales as 1 / theta).
__host__ __device__ inline double dcov_eval(const CovDev& c, double hx, double hy) {
  return c.sigma2 * matern_g(c.nu_code, lag_x(c, hx, hy)) / c.theta;
}

// C(h) and dC(h)/dtheta together.  For nu = 1 in the quadrature regime the
// two sums share their exponentials (t K_1 keeps the operation order of
// t_bessel_k1; t^2 K_0 is rounded differently from t2_bessel_k0).
__host__ __device__ inline void cov_dcov_eval(const CovDev& c, double hx, double hy, double& cv,
                                              double& dv) {
  const double x = lag_x(c, hx, hy);
  if (c.nu_code == 1) {
    const double t = kSqrt2 * x;
    if (t > 2.0 && t <= 30.0) {
      double s1 = 0.5, s0 = 0.5;
#pragma unroll 4
      for (int j = 1; j < 32; ++j) {
        const double ch = cosh_eighth(j);
        const double e = exp(-t * (ch - 1.0));
        s1 += e * ch;
        s0 += e;
      }
      const double f = t * exp(-t) * 0.125;
      cv = c.sigma2 * (f * s1);
      dv = c.sigma2 * (t * f * s0) / c.theta;
      return;
    }
  }
  cv = c.sigma2 * matern_rho(c.nu_code, x);
  dv = c.sigma2 * matern_g(c.nu_code, x) / c.theta;
}

// FP32 correlation from a pre-scaled lag length for the mixed-precision
// cross-covariance: the caller scales coordinates so that xs = kappa * x with
// kappa = log2(e) (nu = 1/2), sqrt(3) (nu = 3/2) or sqrt(2) (nu = 1).
__device__ inline float rho_scaled_f32(int nu_code, float xs) {
  if (nu_code == 0) return __builtin_amdgcn_exp2f(-xs);
  if (nu_code == 2) return (1.0f + xs) * __builtin_amdgcn_exp2f(-xs * (float)kLog2e);
  // nu = 1: xs = t; same series / quadrature as the FP64 routine, in FP32.
  const float t = xs;
  if (t <= 0.0f) return 1.0f;
  if (t <= 2.0f) {
    const float q = 0.25f * t * t;
    float f = 1.0f, si = 0.0f, sp = 0.0f, psi1 = -(float)kEuler;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      const float psi2 = psi1 + 1.0f / (float)(k + 1);
      si += f;
      sp += (psi1 + psi2) * f;
      f *= q / (float)((k + 1) * (k + 2));
      psi1 = psi2;
    }
    return 1.0f + 2.0f * q * (__builtin_amdgcn_logf(0.5f * t) * 0.69314718f) * si - q * sp;
  }
  float s = 0.5f;
#pragma unroll
  for (int j = 2; j < 32; j += 2) {               // step 1/4 suffices in FP32
    const float c = (float)cosh_eighth(j);
    s += __builtin_amdgcn_exp2f(-t * (c - 1.0f) * (float)kLog2e) * c;
  }
  return t * __builtin_amdgcn_exp2f(-t * (float)kLog2e) * 0.25f * s;
}

// ------------------------------------------------------------------- Philox
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 32x32->64 multiplications with the Weyl-sequence key schedule.
struct u32x4 { uint32_t x, y, z, w; };

__host__ __device__ inline u32x4 philox4x32_10(u32x4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
    const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
    const u32x4 o = {(uint32_t)(p1 >> 32) ^ c.y ^ k0, (uint32_t)p1,
                     (uint32_t)(p0 >> 32) ^ c.w ^ k1, (uint32_t)p0};
    c = o;
  }
  return c;
}

// Uniform (x + 1/2) 2^-32 and Box-Muller on word pairs: words (0,1) give
// normals 0,1 and words (2,3) give normals 2,3 of a block.
__host__ __device__ inline double u01_f64(uint32_t x) {
  return ((double)x + 0.5) * 2.3283064365386962890625e-10;
}

__device__ inline void box_muller_f64(uint32_t a, uint32_t b, double& z0, double& z1) {
  const double rad = sqrt(-2.0 * log(u01_f64(a)));
  double s, c;
  sincospi(2.0 * u01_f64(b), &s, &c);
  z0 = rad * c;
  z1 = rad * s;
}

// FP32 variant for the mixed path: hardware log2 and sin/cos taking their
// argument in revolutions (sin(2 pi u) directly).
__device__ inline void box_muller_f32(uint32_t a, uint32_t b, float& z0, float& z1) {
  const float ua = __builtin_fmaf((float)a, 2.3283064365386963e-10f, 1.1641532182693481e-10f);
  const float ub = __builtin_fmaf((float)b, 2.3283064365386963e-10f, 1.1641532182693481e-10f);
  const float rad = __builtin_amdgcn_sqrtf(-1.3862943611198906f * __builtin_amdgcn_logf(ua));
  z0 = rad * __builtin_amdgcn_cosf(ub);
  z1 = rad * __builtin_amdgcn_sinf(ub);
}

// Key and counter words of one call's noise: realization r of the call uses
// counter word 1 = first + (*roff when roff is given) + r and word 2 = event.
// roff lets a captured launch sequence be replayed for later realizations
// by rewriting one device integer.
struct NoiseKey {
  uint32_t k0, k1;
  int first;
  uint32_t event;
  const int* roff;
  __device__ __forceinline__ int base() const { return first + (roff ? *roff : 0); }
};

// Four normals of block `blk` of (realization r, event, stream).
__device__ inline void normals4_f64(uint32_t k0, uint32_t k1, uint32_t blk, uint32_t r,
                                    uint32_t event, uint32_t stream, double z[4]) {
  const u32x4 w = philox4x32_10({blk, r, event, stream}, k0, k1);
  box_muller_f64(w.x, w.y, z[0], z[1]);
  box_muller_f64(w.z, w.w, z[2], z[3]);
}

__device__ inline void normals4_f32(uint32_t k0, uint32_t k1, uint32_t blk, uint32_t r,
                                    uint32_t event, uint32_t stream, float z[4]) {
  const u32x4 w = philox4x32_10({blk, r, event, stream}, k0, k1);
  box_muller_f32(w.x, w.y, z[0], z[1]);
  box_muller_f32(w.z, w.w, z[2], z[3]);
}

}  // namespace cesim
