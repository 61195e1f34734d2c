"""Nearest-neighbour Kriging (oracle side; test infrastructure only).

Section 2.2 moves the information of the off-grid observations onto grid
nodes: every observation's n_p order neighbourhood (the same (2 n_p)^2
nearest nodes as the local-Kriging window of Section 2.1, clamped inside the
grid) becomes a set of surrogate observation sites, overlapping
neighbourhoods merged, so n_N <= n (2 n_p)^2 sites, taken here in ascending
node index.  Section 3.2 gives the surrogate problem:

    z_N       = K_N2 (K22 + tau^2 I)^{-1} z        (Kriging from all the data)
    sigma_N^2 = diag(K_NN - K_N2 (K22 + tau^2 I)^{-1} K_2N)
    z*        = y(S_N) + eps*,   eps*_j ~ N(0, tau^2 + sigma_N,j^2),

with N the surrogate sites and 2 the observations (the printed weight
formula swaps the grid and observation subscripts, and the printed error
variance leaves tau^2 out of the inverse; both readings are listed with the
method's other readings: the error variance taken is that of the predictor
z_N actually uses, i.e. with tau^2, and ``sigma_without_nugget`` switches to
the printed form).  The conditional simulation then runs on the grid with
the surrogate data and a per-site nugget:

    B_r = (K_NN + tau^2 I + Sigma_N)^{-1} (z_N - z*_r),   v_r = y_r + K_1N B_r,

and the variance it realizes at grid node g (Section 3.2) is

    SE_N(g)^2 = C(0) - K_gN (K_NN + tau^2 I + Sigma_N)^{-1} K_Ng.

Pins (tests/test_oracle_nnkrige.py): SE_N^2 against the diagonal of the
covariance of the composed linear map of the whole nearest-neighbour
simulation; the surrogate sites against a brute-force nearest-node search;
z_N and sigma_N^2 reduce to the data and tau^2-free zeros for noise-free
observations on nodes; the Monte Carlo variance of the simulation; listed
nodes against the full grid; mse_nn at least SE_E (optimality of exact
Kriging).
"""

import numpy as np
from scipy.linalg import cho_factor, cho_solve

from . import ce, kriging, localkrige, philox
from .covariance import Cov, cross_covariance


def surrogate_sites(obs_xy, grid, k):
    """Flattened node indices (x fastest) of the merged neighbourhoods, sorted."""
    npp = int(round(np.sqrt(k))) // 2
    a, b = localkrige.window_corners(obs_xy, grid.x0, grid.y0, grid.dx, grid.dy, grid.m1,
                                     grid.m2, npp)
    p, q = localkrige.window_offsets(npp)
    idx = (b[:, None] + q[None, :]) * grid.m1 + a[:, None] + p[None, :]
    return np.unique(idx.ravel())


def site_xy(grid, idx):
    idx = np.asarray(idx)
    return np.stack([grid.x0 + (idx % grid.m1) * grid.dx, grid.y0 + (idx // grid.m1) * grid.dy],
                    axis=1)


def surrogate(cov: Cov, grid, obs_xy, z, tau2, k, sigma_without_nugget=False):
    """Surrogate sites, their coordinates, the surrogate data z_N and the
    prediction error variances sigma_N^2."""
    obs_xy = np.asarray(obs_xy, dtype=np.float64).reshape(-1, 2)
    idx = surrogate_sites(obs_xy, grid, k)
    xy = site_xy(grid, idx)
    K2N = cross_covariance(obs_xy, xy, cov)
    A = kriging.obs_matrix(obs_xy, cov, tau2)
    X = np.linalg.solve(A, K2N)                                  # A^{-1} K_2N
    zN = X.T @ np.asarray(z, dtype=np.float64)
    if sigma_without_nugget:
        X0 = np.linalg.solve(kriging.obs_matrix(obs_xy, cov, 0.0), K2N)
        s2 = cov.sigma2 - np.sum(K2N * X0, axis=0)
    else:
        s2 = cov.sigma2 - np.sum(K2N * X, axis=0)
    return dict(idx=idx, xy=xy, zN=zN, sigmaN2=np.maximum(s2, 0.0))


def surrogate_factor(cov: Cov, xy, tau2, sigmaN2):
    """Cholesky factor of K_NN + tau^2 I + Sigma_N."""
    A = kriging.obs_matrix(xy, cov, tau2 + np.asarray(sigmaN2))
    try:
        return cho_factor(A, lower=True)
    except np.linalg.LinAlgError as e:
        raise kriging.NotPositiveDefinite(str(e))


def se_nn(cov: Cov, grid, obs_xy, tau2, k, rows=None, sigma_without_nugget=False):
    """SE_N on the grid (flattened, x fastest), or on the nodes listed in rows."""
    s = surrogate(cov, grid, obs_xy, np.zeros(len(obs_xy)), tau2, k, sigma_without_nugget)
    fac = surrogate_factor(cov, s["xy"], tau2, s["sigmaN2"])
    G = grid.points() if rows is None else grid.points()[np.asarray(rows)]
    KgN = cross_covariance(G, s["xy"], cov)
    return np.sqrt(np.maximum(cov.sigma2 - np.sum(KgN * cho_solve(fac, KgN.T).T, axis=1), 0.0))


def conditional_simulation_nn(cov: Cov, grid, obs_xy, z, tau2, k, seed, nreal, first_real=0,
                              t1=None, t2=None, event=0):
    """Nearest-neighbour conditional simulation for realizations first_real ..
    first_real + nreal - 1: the CE draw, the surrogate synthetic data
    z*_r = y_r(S_N) + sqrt(tau^2 + sigma_N^2) xi_r (xi_r[j]: the stream-1
    normal of surrogate site j), and v_r = y_r + K_1N B_r."""
    from .pipeline import setup
    s = surrogate(cov, grid, obs_xy, z, tau2, k)
    t1, t2, sl, info = setup(cov, grid, t1, t2)
    reals = np.arange(first_real, first_real + nreal)
    y = ce.ce_draw(sl, seed, reals, grid.m1, grid.m2, event)
    nN = s["idx"].size
    xi = philox.offgrid_noise(seed, nN, reals, event)
    zstar = y.reshape(nreal, -1)[:, s["idx"]] + np.sqrt(tau2 + s["sigmaN2"])[None, :] * xi
    fac = surrogate_factor(cov, s["xy"], tau2, s["sigmaN2"])
    B = kriging.coefficients(fac, s["zN"], zstar)
    v = kriging.condition_fields(y, B, s["xy"], cov, grid.x0, grid.y0, grid.dx, grid.dy,
                                 grid.m1, grid.m2)
    return dict(t1=t1, t2=t2, y=y, xi=xi, zstar=zstar, B=B, v=v, **s)


def linear_map_nn(cov: Cov, grid, obs_xy, tau2, k, t1=None, t2=None):
    """(Me, Mx) with v - E v = Me [eps_{2P}; eps_{2P+1}] + Mx xi for the
    nearest-neighbour simulation, realization 2P of a pair (the data enter
    only the mean).  Tiny problems only."""
    from .pipeline import draw_matrix, setup
    s = surrogate(cov, grid, obs_xy, np.zeros(len(obs_xy)), tau2, k)
    t1, t2, sl, _ = setup(cov, grid, t1, t2)
    Bce = draw_matrix(sl, grid.m1, grid.m2)                      # (M, 2N)
    fac = surrogate_factor(cov, s["xy"], tau2, s["sigmaN2"])
    nN = s["idx"].size
    K1N = cross_covariance(grid.points(), s["xy"], cov)
    P = K1N @ cho_solve(fac, np.eye(nN))                         # K_1N (...)^{-1}
    J = np.zeros((nN, grid.m1 * grid.m2))
    J[np.arange(nN), s["idx"]] = 1.0
    Me = Bce - P @ J @ Bce
    Mx = -P * np.sqrt(tau2 + s["sigmaN2"])[None, :]
    return Me, Mx


def mse_nn(cov: Cov, grid, obs_xy, tau2, k):
    """Root mean-square error of the nearest-neighbour Kriging predictor
    K_gN F^{-1} z_N (F = K_NN + tau^2 I + Sigma_N, z_N = K_N2 A^{-1} z) as a
    predictor of y(g) from the real data: with u_g = K_2N F^{-1} K_Ng,
        MSE(g) = C(0) - 2 u_g . A^{-1} K_2g + u_g . A^{-1} u_g.
    Not the variance the simulation realizes (se_nn): an alternative reading
    of what Table 2 scores, kept for the comparison of readings."""
    obs_xy = np.asarray(obs_xy, dtype=np.float64).reshape(-1, 2)
    s = surrogate(cov, grid, obs_xy, np.zeros(len(obs_xy)), tau2, k)
    fac = surrogate_factor(cov, s["xy"], tau2, s["sigmaN2"])
    G = grid.points()
    U = cho_solve(fac, cross_covariance(s["xy"], G, cov)).T @ cross_covariance(s["xy"], obs_xy, cov)
    A = kriging.obs_matrix(obs_xy, cov, tau2)
    Kg2 = cross_covariance(G, obs_xy, cov)
    AiU = np.linalg.solve(A, U.T).T
    v = cov.sigma2 - 2.0 * np.sum(AiU * Kg2, axis=1) + np.sum(AiU * U, axis=1)
    return np.sqrt(np.maximum(v, 0.0))
