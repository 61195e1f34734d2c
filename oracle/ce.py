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
* Draw, two realizations per transform (the complex form of the CE draw:
  Dietrich and Newsam, SIAM J. Sci. Comput. 18, 1997; Wood and Chan
  generate the transformed noise directly in the same way).  Realizations
  2P and 2P + 1 form pair P.  With eps_{2P}, eps_{2P+1} two T2 x T1 fields
  of iid N(0, 1) (Philox stream 0) and zeta_P = eps_{2P} + i eps_{2P+1},
      W_P = FFT2(sqrt(lambda / N) * zeta_P),     N = T1 T2,
  (unnormalised forward transform) and y_{2P} = Re W_P, y_{2P+1} = Im W_P,
  each cropped to [0:m2, 0:m1].  Why this is exact: with F the DFT matrix,
  E[W W^*] = (2/N) F diag(lambda) F^* = 2 C_torus (lambda real and even) and
  E[W W^T] = 0 because E[zeta zeta^T] = I - I = 0; so Re W and Im W each
  have covariance C_torus, whose crop is [C(g - g')], and they are
  uncorrelated, hence independent.  One 2D FFT serves two realizations.

Pins (tests/test_oracle_ce.py): brute-force DFT on tiny tori, trace
sum(lambda) = N C(0), evenness, and the exactness of the draw: the explicit
linear maps B_re, B_im from the pair's noise (eps_{2P}, eps_{2P+1}) to its
two fields satisfy B_re B_re^T = B_im B_im^T = [C(g - g')] and
B_re B_im^T = 0 on small grids, including padded and anisotropic cases.
"""

import numpy as np

from . import philox
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


def ce_draw_pair(sqrt_lam, eps_even, eps_odd, m1, m2):
    """Both fields of one pair: W = FFT2(sqrt(lambda / N) (eps_even + i
    eps_odd)) cropped to the grid; returns (Re W, Im W), each (m2, m1)."""
    t2, t1 = sqrt_lam.shape
    w = np.fft.fft2((sqrt_lam / np.sqrt(t1 * t2)) * (np.asarray(eps_even, dtype=np.float64)
                                                    + 1j * np.asarray(eps_odd, dtype=np.float64)))
    return w.real[:m2, :m1].copy(), w.imag[:m2, :m1].copy()


def ce_draw(sqrt_lam, seed, reals, m1, m2, event=0):
    """Unconditional fields y_r, shape (len(reals), m2, m1), for the absolute
    realization indices ``reals``: y_r = Re W_P (r even) or Im W_P (r odd)
    of pair P = r // 2, whose noise is eps_{2P} + i eps_{2P+1} (Philox
    stream 0, counter word 2 = event)."""
    t2, t1 = sqrt_lam.shape
    reals = [int(r) for r in reals]
    out = np.empty((len(reals), m2, m1))
    pair, fields = None, None
    for i, r in enumerate(reals):
        P = r // 2
        if P != pair:
            eps = philox.torus_noise(seed, t1, t2, [2 * P, 2 * P + 1], event)
            pair, fields = P, ce_draw_pair(sqrt_lam, eps[0], eps[1], m1, m2)
        out[i] = fields[r % 2]
    return out
