"""Gradient of a linear ensemble statistic of the conditional realizations
with respect to the range, the sill, the nugget and the observed values
(oracle side; test infrastructure only: an FP64 reference adjoint).

The statistic is
    L = (1/R) sum_r sum_g w_g v_r[g]
over the conditional fields v_r of Section 2 (steps 1-5, with the local
Kriging of Section 2.1 for steps 2-4) and fixed grid weights w.  Each v_r is
affine in its noise (the pair noise zeta_P = eps_{2P} + i eps_{2P+1} of the
circulant-embedding draw, P = r // 2, and xi_r for the nugget of the
synthetic data): y_r = Re(c_r W_P) with W_P = FFT2(sqrt(lambda / N) zeta_P),
c_r = 1 for even r and -i for odd r.  So L equals the same expression
evaluated once on the mean noises zeta_bar = mean_r c_r zeta_{r // 2}
(complex) and xi_bar = mean_r xi_r:
    ybar   = crop(Re FFT2(sqrt(lambda / N) zeta_bar))      (Section 2, step 2)
    zbar*  = W1 ybar + phi * xi_bar                        (Section 2.1 (b)-(c))
    L      = w . ybar + u . (z - zbar*),  u = A^{-1} K21 w (steps 1, 4, 5; eq. (4))
with A = K22 + tau^2 I and phi_i = sqrt(tau^2 + gamma_i).

Differentiating that expression with dA^{-1} = -A^{-1} dA A^{-1} and
cbar = A^{-1}(z - zbar*), p = K21 w:
    dL = w . dybar + dp . cbar - u . dA cbar - u . dzbar* + u . dz
    dzbar*_i = dw_i . ybar[N_i] + w_i . dybar[N_i] + xi_bar_i dphi_i
per parameter:
  z      : dL/dz = u.
  tau^2  : dA = I, dphi_i = 1 / (2 phi_i); nothing else moves.
  sigma^2: C is proportional to sigma^2, so sqrt(lambda) and ybar scale by
           sigma (dybar = ybar / (2 sigma^2)), dp = p / sigma^2,
           dA = K22 / sigma^2, dw = 0, dgamma = gamma / sigma^2.
  theta  : every covariance moves: dC/dtheta = sigma^2 g(x) / theta with
           x = d / theta and g(x) = -x rho'(x); dlambda = Re FFT2(dc) of the
           torus base, d sqrt(lambda) = dlambda / (2 sqrt(lambda)) (set to 0
           where lambda <= 1e-12 lambda_max, as the setup clamps there);
           dw_i = K11^{-1}(dk_i - dK11 w_i); dgamma_i = -2 dk_i . w_i + w_i . dK11 w_i.

g(x) for the Matern family of Section 3.3: with t = sqrt(2 nu) x and
d/dt [t^nu K_nu(t)] = -t^nu K_{nu-1}(t) (Abramowitz and Stegun 9.6.28),
    g(x) = 2^(1-nu) / Gamma(nu) t^(nu+1) K_{nu-1}(t),
i.e. x e^-x (nu = 1/2), t^2 K_0(t) (nu = 1), 3 x^2 e^(-sqrt(3) x) (nu = 3/2).

Pins (tests/test_oracle_gradient.py): g agrees with central differences of
the correlation and the closed forms with the Bessel form; L from the mean
noises equals the ensemble statistic of the full simulation; every gradient
component agrees with central finite differences (h = 1e-6, common random
numbers) of the ensemble statistic of the full simulation.
"""

import numpy as np
from scipy.linalg import cho_factor, cho_solve
from scipy.special import gamma as gamma_fn
from scipy.special import kv

from . import ce, kriging, localkrige, philox
from .covariance import Cov, covariance, cross_covariance, lag_distance


def matern_g(x, nu):
    """g(x) = -x rho_nu'(x), so that dC/dtheta = sigma^2 g(d / theta) / theta."""
    x = np.asarray(x, dtype=np.float64)
    if nu == 0.5:
        return x * np.exp(-x)
    if nu == 1.5:
        return 3.0 * x * x * np.exp(-np.sqrt(3.0) * x)
    return matern_g_bessel(x, nu)


def matern_g_bessel(x, nu):
    """The Bessel form 2^(1-nu) / Gamma(nu) t^(nu+1) K_{nu-1}(t), t = sqrt(2 nu) x."""
    x = np.asarray(x, dtype=np.float64)
    t = np.sqrt(2.0 * nu) * x
    out = np.zeros_like(t)
    pos = t > 0
    tp = t[pos]
    out[pos] = (2.0 ** (1.0 - nu) / gamma_fn(nu)) * tp ** (nu + 1.0) * kv(nu - 1.0, tp)
    return out


def dcov_dtheta(hx, hy, cov: Cov):
    """dC(h)/dtheta for lag components hx, hy."""
    d = lag_distance(hx, hy, cov)
    return cov.sigma2 * matern_g(d / cov.range, cov.nu) / cov.range


def cross_dcov(p, q, cov: Cov):
    p = np.asarray(p, dtype=np.float64).reshape(-1, 2)
    q = np.asarray(q, dtype=np.float64).reshape(-1, 2)
    return dcov_dtheta(p[:, 0:1] - q[None, :, 0], p[:, 1:2] - q[None, :, 1], cov)


def torus_base_dtheta(cov: Cov, dx, dy, t1, t2):
    """dc/dtheta of the torus base, with the Nyquist lines averaged over the
    sign of the lag as in the base itself."""
    hx = ce.wrapped_lags(t1).astype(np.float64) * dx
    hy = ce.wrapped_lags(t2).astype(np.float64) * dy
    HX, HY = np.meshgrid(hx, hy)
    c = dcov_dtheta(HX, HY, cov)
    if t1 % 2 == 0:
        q1 = t1 // 2
        c[:, q1] = 0.5 * (dcov_dtheta(hx[q1], hy, cov) + dcov_dtheta(-hx[q1], hy, cov))
    if t2 % 2 == 0:
        q2 = t2 // 2
        c[q2, :] = 0.5 * (dcov_dtheta(hx, hy[q2], cov) + dcov_dtheta(hx, -hy[q2], cov))
    if t1 % 2 == 0 and t2 % 2 == 0:
        q1, q2 = t1 // 2, t2 // 2
        c[q2, q1] = 0.5 * (dcov_dtheta(hx[q1], hy[q2], cov) + dcov_dtheta(hx[q1], -hy[q2], cov))
    return c


def mean_noises(seed, t1, t2, n, reals, event=0, chunk=16):
    """zeta_bar (t2, t1), complex, and xi_bar (n,) over the realizations
    ``reals``: zeta_bar = mean_r c_r (eps_{2P} + i eps_{2P+1}), P = r // 2,
    c_r = 1 (r even) or -i (r odd)."""
    reals = [int(r) for r in reals]
    eb = np.zeros((t2, t1), dtype=np.complex128)
    xb = np.zeros(n)
    for r in reals:
        P = r // 2
        eps = philox.torus_noise(seed, t1, t2, [2 * P, 2 * P + 1], event)
        zeta = eps[0] + 1j * eps[1]
        eb += zeta if r % 2 == 0 else -1j * zeta
    for i in range(0, len(reals), chunk):
        xb += philox.offgrid_noise(seed, n, reals[i:i + chunk], event).sum(axis=0)
    return eb / len(reals), xb / len(reals)


def local_krige_dtheta(obs_xy, cov: Cov, grid, k):
    """Window corners, weights, gamma and their theta-derivatives
    (Section 2.1 (b); Section 3.1's W1 and gamma)."""
    npp = int(round(np.sqrt(k))) // 2
    a, b, W, gamma = localkrige.local_krige(obs_xy, cov, grid.x0, grid.y0, grid.dx, grid.dy,
                                            grid.m1, grid.m2, k)
    p, q = localkrige.window_offsets(npp)
    hx = (p[:, None] - p[None, :]).astype(np.float64) * grid.dx
    hy = (q[:, None] - q[None, :]).astype(np.float64) * grid.dy
    fac = cho_factor(localkrige.window_cov(cov, grid.dx, grid.dy, npp), lower=True)
    dK11 = dcov_dtheta(hx, hy, cov)
    obs_xy = np.asarray(obs_xy, dtype=np.float64).reshape(-1, 2)
    n = obs_xy.shape[0]
    dW = np.empty_like(W)
    dgamma = np.empty(n)
    for i in range(n):
        gx = grid.x0 + (a[i] + p) * grid.dx - obs_xy[i, 0]
        gy = grid.y0 + (b[i] + q) * grid.dy - obs_xy[i, 1]
        dk = dcov_dtheta(gx, gy, cov)
        dW[i] = cho_solve(fac, dk - dK11 @ W[i])
        dgamma[i] = (-2.0 * dk @ W[i] + W[i] @ dK11 @ W[i]) if gamma[i] > 0.0 else 0.0
    return a, b, W, gamma, dW, dgamma


def linear_stat_gradient(cov: Cov, grid, obs_xy, z, tau2, k, seed, nreal, weights, t1, t2,
                         first_real=0, event=0):
    """L and dL/d(theta, sigma^2, tau^2, z) for the realizations
    first_real .. first_real + nreal - 1 on the (t1, t2) torus.
    weights: (m2, m1) grid weights w."""
    obs_xy = np.asarray(obs_xy, dtype=np.float64).reshape(-1, 2)
    z = np.asarray(z, dtype=np.float64)
    w = np.asarray(weights, dtype=np.float64).reshape(grid.m2, grid.m1)
    n = obs_xy.shape[0]
    npp = int(round(np.sqrt(k))) // 2
    s2, th = cov.sigma2, cov.range
    # circulant embedding and its theta-derivative
    lam = np.fft.fft2(ce.torus_base(cov, grid.dx, grid.dy, t1, t2)).real
    dlam = np.fft.fft2(torus_base_dtheta(cov, grid.dx, grid.dy, t1, t2)).real
    s = np.sqrt(np.maximum(lam, 0.0))
    keep = lam > 1e-12 * lam.max()
    ds = np.where(keep, dlam / (2.0 * np.where(keep, s, 1.0)), 0.0)
    eb, xb = mean_noises(seed, t1, t2, n, range(first_real, first_real + nreal), event)
    rn = 1.0 / np.sqrt(t1 * t2)
    ybar = np.fft.fft2(rn * s * eb).real[:grid.m2, :grid.m1]
    dybar = np.fft.fft2(rn * ds * eb).real[:grid.m2, :grid.m1]
    # local Kriging and the mean synthetic data
    a, b, W, gamma, dW, dgamma = local_krige_dtheta(obs_xy, cov, grid, k)
    phi = np.sqrt(tau2 + gamma)
    if tau2 == 0.0 and np.any(gamma <= 1e-12 * cov.sigma2):
        # tau^2 = 0 and gamma_i = 0 (a station on a grid node, where gamma_i
        # is 0 up to round-off): dphi_i/dtau^2 = 1 / (2 phi_i) is unbounded
        raise ValueError("dL/dtau^2 does not exist: zero nugget and a station with gamma_i = 0")
    wy = np.einsum("nk,nk->n", localkrige.gather_windows(ybar, a, b, npp), W)
    dwy = np.einsum("nk,nk->n", localkrige.gather_windows(ybar, a, b, npp), dW)
    wdy = np.einsum("nk,nk->n", localkrige.gather_windows(dybar, a, b, npp), W)
    zbar = wy + phi * xb
    # Kriging system and the cross-covariance products
    fac = kriging.factor(obs_xy, cov, tau2)
    gp = grid.points()
    wf = w.reshape(-1)
    p = np.zeros(n)
    dp = np.zeros(n)
    for g0 in range(0, gp.shape[0], 8192):          # K21 w in blocks of grid nodes
        p += cross_covariance(obs_xy, gp[g0:g0 + 8192], cov) @ wf[g0:g0 + 8192]
        dp += cross_dcov(obs_xy, gp[g0:g0 + 8192], cov) @ wf[g0:g0 + 8192]
    u = cho_solve(fac, p)
    bvec = z - zbar
    cbar = cho_solve(fac, bvec)
    dK22 = cross_dcov(obs_xy, obs_xy, cov)
    L = float(np.sum(w * ybar) + u @ bvec)
    d_tau2 = float(-u @ cbar - np.sum(u * xb / (2.0 * phi)))
    d_sigma2 = float(np.sum(w * ybar) / (2.0 * s2) + p @ cbar / s2
                     - (u @ bvec - tau2 * (u @ cbar)) / s2
                     - np.sum(u * (wy / (2.0 * s2) + xb * gamma / (2.0 * s2 * phi))))
    d_theta = float(np.sum(w * dybar) + dp @ cbar - u @ (dK22 @ cbar)
                    - np.sum(u * (dwy + wdy + xb * dgamma / (2.0 * phi))))
    return dict(L=L, d_range=d_theta, d_sigma2=d_sigma2, d_tau2=d_tau2, d_z=u,
                ybar=ybar, dybar=dybar, zbar=zbar, u=u, cbar=cbar, p=p, dp=dp,
                zeta_bar=eb, xi_bar=xb)


def fields_vjp(cov: Cov, grid, obs_xy, z, tau2, k, seed, vbar, t1, t2, first_real=0, event=0):
    """The vector-Jacobian product of the conditional fields: for vbar (R, m2,
    m1), the derivatives of a statistic with respect to v_r of realizations
    first_real .. first_real + R - 1, returns sum_r vbar[r] . v_r and
    sum_r vbar[r] . dv_r/d(theta, sigma^2, tau^2, z).  Each v_r is affine in
    its own noise, so this is the sum over r of the linear statistic of
    realization r alone (nreal = 1) with weights vbar[r]."""
    vbar = np.asarray(vbar, dtype=np.float64)
    tot = dict(L=0.0, d_range=0.0, d_sigma2=0.0, d_tau2=0.0, d_z=0.0)
    for r in range(vbar.shape[0]):
        g = linear_stat_gradient(cov, grid, obs_xy, z, tau2, k, seed, 1, vbar[r], t1, t2,
                                 first_real + r, event)
        for key in tot:
            tot[key] = tot[key] + g[key]
    return tot


def ensemble_stat(cov: Cov, grid, obs_xy, z, tau2, k, seed, nreal, weights, t1, t2,
                  first_real=0, event=0):
    """L = (1/R) sum_r sum_g w_g v_r[g] from the full simulation (Section 2)."""
    from .pipeline import conditional_simulation
    out = conditional_simulation(cov, grid, obs_xy, z, tau2, k, seed, nreal, first_real,
                                 t1, t2, event)
    w = np.asarray(weights, dtype=np.float64).reshape(grid.m2, grid.m1)
    return float(np.mean(np.sum(out["v"] * w[None], axis=(1, 2))))
