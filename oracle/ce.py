"""Circulant embedding: torus setup and the unconditional grid draw (oracle
side; test infrastructure only).

Section 1 introduces circulant embedding (CE) as the fast, exact simulator of
a stationary Gaussian field on a regular m x m grid, costing one FFT of the
2m x 2m torus ("40 m^2 log2 2m" operations); Section 2.1 item (a) uses it for
the grid field y(S^g).  The paper does not spell the algorithm out; this is
the textbook construction it cites (Wood and Chan; Chan and Wood):

* Grid (Section 2): nodes g_ij = (x0 + i dx, y0 + j dy), 0 <= i < m1,
  0 <= j < m2; fields are stored [j][i] (x fastest).
* Torus base: c[q2, q1] = C(w(q1) dx, w(q2) dy) with the wrapped lag
  w(q) = q for q <= T/2 and q - T otherwise.  On a Nyquist line (q = T/2,
  T even) the two signed lags +-T/2 are the same torus point; for an
  anisotropic C they give different values, so the average over the sign of
  that component is used, which keeps c even and its spectrum real.  Lags
  used inside the m x m crop never reach T/2, so the crop covariance is
  unaffected.
* Eigenvalues: lambda = Re FFT2(c) (unnormalised).  The embedding is accepted
  when min(lambda) >= -1e-12 max(lambda), the imaginary parts are round-off
  (at most 1e-12 max(lambda)) and sum(lambda) = N C(0) to 1e-9 relative;
  remaining tiny negatives are clamped to 0.  Otherwise the next torus size on the ladder is tried:
  T = S(f m) for f in (2, 3, 4, 6, 8), where S(n) is the smallest integer
  >= n whose only prime factors are 2, 3 and 5 (the sizes the FFT handles).
* Draw: y = Re(IFFT2(sqrt(lambda) * FFT2(eps)))[0:m2, 0:m1] with eps a
  T2 x T1 field of iid N(0, 1) (Philox stream 0) and IFFT2 including
  1 / (T1 T2).  Because lambda is real and even, the map eps -> y is real;
  two realizations may therefore share one complex transform (real and
  imaginary parts), which the HIP path does and this oracle does not need.

Pins (tests/test_oracle_ce.py): brute-force DFT on tiny tori, trace
sum(lambda) = N C(0), evenness, and the exactness of the draw: the explicit
linear map B of the draw satisfies B B^T = [C(g - g')] on small grids,
including padded and anisotropic cases.
"""

import numpy as np

from .covariance import Cov, covariance

LADDER_FACTORS = (2, 3, 4, 6, 8)
MAX_TORUS = 8192
NEG_TOL = 1e-12


def is_smooth(n):
    for p in (2, 3, 5):
        while n % p == 0:
            n //= p
    return n == 1


def next_smooth(n):
    n = max(int(n), 1)
    while not is_smooth(n):
        n += 1
    return n


def torus_ladder(m1, m2):
    """Candidate (T1, T2) pairs, in the order they are tried."""
    out = []
    for f in LADDER_FACTORS:
        t1, t2 = next_smooth(f * m1), next_smooth(f * m2)
        if t1 > MAX_TORUS or t2 > MAX_TORUS:
            break
        if not out or out[-1] != (t1, t2):
            out.append((t1, t2))
    return out


def wrapped_lags(t):
    q = np.arange(t)
    return np.where(q <= t // 2, q, q - t)


def torus_base(cov: Cov, dx, dy, t1, t2):
    """c[q2, q1] = C(w(q1) dx, w(q2) dy), Nyquist lines averaged over sign."""
    hx = wrapped_lags(t1).astype(np.float64) * dx
    hy = wrapped_lags(t2).astype(np.float64) * dy
    HX, HY = np.meshgrid(hx, hy)            # shape (t2, t1)
    c = covariance(HX, HY, cov)
    if t1 % 2 == 0:
        q1 = t1 // 2
        c[:, q1] = 0.5 * (covariance(hx[q1], hy, cov)
                          + covariance(-hx[q1], hy, cov))
    if t2 % 2 == 0:
        q2 = t2 // 2
        c[q2, :] = 0.5 * (covariance(hx, hy[q2], cov)
                          + covariance(hx, -hy[q2], cov))
    if t1 % 2 == 0 and t2 % 2 == 0:
        q1, q2 = t1 // 2, t2 // 2
        c[q2, q1] = 0.5 * (covariance(hx[q1], hy[q2], cov)
                           + covariance(hx[q1], -hy[q2], cov))
    return c


def eigenvalues(c):
    """lambda = Re FFT2(c) and the check quantities of the setup."""
    f = np.fft.fft2(c)
    lam = f.real.copy()
    info = dict(lam_min=float(lam.min()), lam_max=float(lam.max()),
                lam_sum=float(lam.sum()),
                max_imag=float(np.abs(f.imag).max()),
                trace=float(c.size * c[0, 0]))
    return lam, info


TRACE_TOL = 1e-9


def accept(info):
    """The spectrum of a valid embedding: lambda_min >= -1e-12 lambda_max;
    real up to round-off (max |Im| <= 1e-12 lambda_max, the base being
    even); and the trace identity sum(lambda) = N c[0, 0] = N C(0) to 1e-9
    relative."""
    return (info["lam_min"] >= -NEG_TOL * info["lam_max"]
            and info["max_imag"] <= NEG_TOL * info["lam_max"]
            and abs(info["lam_sum"] - info["trace"]) <= TRACE_TOL * abs(info["trace"]))


class NegativeEigenvalue(ValueError):
    pass


def ce_setup(cov: Cov, dx, dy, m1, m2, t1=None, t2=None):
    """Choose the torus and return (t1, t2, sqrt_lambda, info).

    With (t1, t2) given, only that torus is tried; otherwise the ladder."""
    cands = [(t1, t2)] if t1 else torus_ladder(m1, m2)
    last = None
    for a, b in cands:
        lam, info = eigenvalues(torus_base(cov, dx, dy, a, b))
        info.update(t1=a, t2=b)
        last = info
        if accept(info):
            return a, b, np.sqrt(np.maximum(lam, 0.0)), info
    raise NegativeEigenvalue(f"no torus on the ladder is non-negative: {last}")


def ce_draw(sqrt_lam, eps, m1, m2):
    """Unconditional fields y_r = Re(IFFT2(s * FFT2(eps_r)))[:m2, :m1].

    eps: (R, T2, T1) real noise; returns (R, m2, m1)."""
    eps = np.asarray(eps, dtype=np.float64)
    single = eps.ndim == 2
    if single:
        eps = eps[None]
    out = np.empty((eps.shape[0], m2, m1))
    for r in range(eps.shape[0]):
        f = np.fft.ifft2(sqrt_lam * np.fft.fft2(eps[r]))
        out[r] = f.real[:m2, :m1]
    return out[0] if single else out
