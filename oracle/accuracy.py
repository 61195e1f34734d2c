"""Prediction standard errors on the grid: exact Kriging and the local-Kriging
approximation (oracle side; test infrastructure only).

Section 3 (eq. (4)): the exact conditional variance of y(g) given the data is
    SE_E(g)^2 = C(0) - K12[g] (K22 + tau^2 I)^{-1} K21[g].
Section 3.1: under local Kriging the grid values predicted in step 4 are
    yhat*  = Lambda y(S^g) + W2 eps*,   Lambda = W2 W1,  W2 = K12 (K22 + tau^2 I)^{-1},
with eps* independent of y(S^g) and Var(eps*_i) = phi_i^2 = tau^2 + gamma_i,
so the approximate prediction variance is the diagonal of
    (Lambda - I) K11 (Lambda - I)^T + W2 diag(phi^2) W2^T.
W1 is sparse (row i: the k weights on the window of s_i), which gives per
grid node g, with W2_g the g-th row of W2:
    SE_L(g)^2 = W2_g Q W2_g^T - 2 W2_g (W1 K11)[:, g] + C(0) + sum_i W2_gi^2 phi_i^2,
    Q = W1 K11 W1^T  (n x n).
Section 3.4 scores SE_L against SE_E by the fraction of grid nodes where the
two agree to three significant figures (Table 1); reading: both rounded to
three significant figures are equal.

Pins (tests/test_oracle_accuracy.py): SE_E^2 against the diagonal of the
exact conditional covariance; SE_L^2 against the diagonal of the covariance
of the whole simulation's linear map (an independent route through steps
1-5); SE_L = SE_E for observations on grid nodes; the rounding to three
significant figures against Python's decimal formatting.
"""

import numpy as np

from . import localkrige
from .covariance import Cov, cross_covariance


def se_exact(cov: Cov, grid, obs_xy, tau2, rows=None):
    """SE_E on the grid (flattened, x fastest), or on the nodes listed in rows."""
    obs_xy = np.asarray(obs_xy, dtype=np.float64).reshape(-1, 2)
    n = obs_xy.shape[0]
    A = cross_covariance(obs_xy, obs_xy, cov) + tau2 * np.eye(n)
    G = grid.points() if rows is None else grid.points()[np.asarray(rows)]
    K12 = cross_covariance(G, obs_xy, cov)
    W2 = np.linalg.solve(A, K12.T).T
    return np.sqrt(cov.sigma2 - np.sum(W2 * K12, axis=1))


def se_local(cov: Cov, grid, obs_xy, tau2, k, rows=None):
    """SE_L on the grid from the closed form of Section 3.1, or on the nodes
    listed in rows (W1 K11 is then formed only on the columns it needs: the
    listed nodes and the window nodes)."""
    obs_xy = np.asarray(obs_xy, dtype=np.float64).reshape(-1, 2)
    n = obs_xy.shape[0]
    G = grid.points()
    rows = np.arange(G.shape[0]) if rows is None else np.asarray(rows)
    A = cross_covariance(obs_xy, obs_xy, cov) + tau2 * np.eye(n)
    W2 = np.linalg.solve(A, cross_covariance(G[rows], obs_xy, cov).T).T  # rows x n
    a, b, W, gamma = localkrige.local_krige(obs_xy, cov, grid.x0, grid.y0, grid.dx, grid.dy,
                                            grid.m1, grid.m2, k)
    npp = int(round(np.sqrt(k))) // 2
    p, q = localkrige.window_offsets(npp)
    idx = np.zeros((n, k), dtype=np.int64)
    for i in range(n):
        idx[i] = (b[i] + q) * grid.m1 + a[i] + p
    cols, inv = np.unique(np.concatenate([rows, idx.ravel()]), return_inverse=True)
    at_rows, at_idx = inv[:rows.size], inv[rows.size:].reshape(n, k)
    W1K = np.zeros((n, cols.size))                                       # (W1 K11)[:, cols]
    for i in range(n):
        nodes = np.stack([grid.x0 + (a[i] + p) * grid.dx, grid.y0 + (b[i] + q) * grid.dy], axis=1)
        W1K[i] = W[i] @ cross_covariance(nodes, G[cols], cov)
    Q = np.stack([W1K[:, at_idx[j]] @ W[j] for j in range(n)], axis=1)   # W1 K11 W1^T
    phi2 = tau2 + gamma
    v = (np.sum((W2 @ Q) * W2, axis=1) - 2.0 * np.sum(W2 * W1K[:, at_rows].T, axis=1)
         + cov.sigma2 + (W2 * W2) @ phi2)
    return np.sqrt(np.maximum(v, 0.0))


def round_sig(x, digits=3):
    x = np.asarray(x, dtype=np.float64)
    e = np.floor(np.log10(np.abs(x)))
    s = 10.0 ** (e - (digits - 1))
    return np.round(x / s) * s


def fraction_sig3(se_l, se_e):
    """Fraction of nodes where SE_L and SE_E agree to three significant figures."""
    return float(np.mean(round_sig(se_l) == round_sig(se_e)))
