"""Local Kriging of off-grid observations from their nearest grid nodes
(oracle side; test infrastructure only).

Section 2.1 approximates steps 2-4 of the conditional simulation: the field
is simulated on the grid by circulant embedding, and each observation value
y(s_i) is then drawn from its conditional law given the (2 n_p)^2 nearest
grid values (item (b)), independently across observations, with nugget
variance phi_i^2 = tau^2 + gamma_i for the synthetic data (item (c)).
Section 3.1 writes the pieces as

    W1 row i   = K21^i (K11^i)^{-1}          (k weights on the window)
    gamma_i    = K22^i - K21^i (K11^i)^{-1} K12^i
    z*         = W1 y(S^g) + eps*,  eps*_i ~ N(0, tau^2 + gamma_i),

where, by role, K11^i is the covariance among the window nodes, K21^i the
covariance between s_i and the window, and K22^i = C(0) (Section 3.6 swaps the
subscripts; the roles are what matter).  Section 3.6 notes that K11^i is the
same matrix for every window of a stationary field.

Neighbourhood (Section 2.1 "order n_p", Section 3.6): 2 n_p nodes per axis,
k = (2 n_p)^2 in all.  The window of s = (sx, sy) starts at
    a = clamp(floor((sx - x0)/dx) - n_p + 1, 0, m1 - 2 n_p)
and likewise b in y, so that an interior point sits in the middle grid box of
its window and a point near the edge keeps a full-size window inside the grid
(the paper pads the grid instead; the clamp keeps the same window size).
Nodes are ordered (a + p, b + q), index alpha = q * 2 n_p + p.

The weights solve K11 w = k_i by Cholesky; gamma_i is clamped at 0.

Joint variant (Section 2.1, last paragraph; Section 3.6): observations in
the same grid box share their window, and their synthetic values can be drawn
jointly from the conditional law given the window,
    z*_G = W1_G y(S^g) + L_G xi_G,  L_G L_G^T = tau^2 I + Gamma_G,
    Gamma_G[i][j] = C(s_i - s_j) - w_i . k_j
(k_j: covariances between the window nodes and s_j), i.e. the diagonal
blocks of the noise matrix become Cholesky factors; a box with one
observation keeps phi_i = sqrt(tau^2 + gamma_i).  A box is the cell
(floor((x - x0)/dx), floor((y - y0)/dy)); members are taken in ascending
index order and xi_G holds their own normals.

Pins (tests/test_oracle_localkrige.py, tests/test_oracle_joint.py): indicator weights and gamma = 0 for
an observation on a node; the window equals the 2 n_p nearest nodes per axis
by brute force; weights and gamma agree with the Schur complement of the joint
covariance; gamma decreases as n_p grows; the full-grid window reproduces the
exact conditional law.
"""

import numpy as np
from scipy.linalg import cho_factor, cho_solve

from .covariance import Cov, covariance


def window_corners(obs_xy, x0, y0, dx, dy, m1, m2, npp):
    """Lower-left node (a, b) of each observation's window: int arrays."""
    obs_xy = np.asarray(obs_xy, dtype=np.float64).reshape(-1, 2)
    i0 = np.floor((obs_xy[:, 0] - x0) / dx).astype(np.int64)
    j0 = np.floor((obs_xy[:, 1] - y0) / dy).astype(np.int64)
    a = np.clip(i0 - npp + 1, 0, m1 - 2 * npp)
    b = np.clip(j0 - npp + 1, 0, m2 - 2 * npp)
    return a, b


def window_offsets(npp):
    """(p, q) offsets of the window nodes in alpha order (q-major)."""
    w = 2 * npp
    q, p = np.divmod(np.arange(w * w), w)
    return p, q


def window_cov(cov: Cov, dx, dy, npp):
    """K11: covariance among the window nodes, from their index lags."""
    p, q = window_offsets(npp)
    hx = (p[:, None] - p[None, :]).astype(np.float64) * dx
    hy = (q[:, None] - q[None, :]).astype(np.float64) * dy
    return covariance(hx, hy, cov)


def local_krige(obs_xy, cov: Cov, x0, y0, dx, dy, m1, m2, k):
    """Returns (a, b, W, gamma): window corners, weights (n, k), gamma (n)."""
    npp = int(round(np.sqrt(k))) // 2
    if (2 * npp) ** 2 != k or npp < 1:
        raise ValueError("k must be (2 n_p)^2")
    if 2 * npp > min(m1, m2):
        raise ValueError("window larger than the grid")
    obs_xy = np.asarray(obs_xy, dtype=np.float64).reshape(-1, 2)
    a, b = window_corners(obs_xy, x0, y0, dx, dy, m1, m2, npp)
    p, q = window_offsets(npp)
    fac = cho_factor(window_cov(cov, dx, dy, npp), lower=True)
    n = obs_xy.shape[0]
    W = np.empty((n, k))
    gamma = np.empty(n)
    c0 = cov.sigma2
    for i in range(n):
        gx = x0 + (a[i] + p) * dx
        gy = y0 + (b[i] + q) * dy
        ki = covariance(gx - obs_xy[i, 0], gy - obs_xy[i, 1], cov)
        w = cho_solve(fac, ki)
        W[i] = w
        gamma[i] = max(0.0, c0 - ki @ w)
    return a, b, W, gamma


def gather_windows(y, a, b, npp):
    """Window values y[b + q, a + p] of each observation: (..., n, k)."""
    p, q = window_offsets(npp)
    rows = b[:, None] + q[None, :]
    cols = a[:, None] + p[None, :]
    return y[..., rows, cols]


def synthetic_obs(y, a, b, W, gamma, tau2, xi):
    """Step 3 under local Kriging: z*_i = W1_i y(S^g) + sqrt(tau^2+gamma_i) xi_i.

    y: (R, m2, m1) grid fields, xi: (R, n) standard normals -> (R, n)."""
    k = W.shape[1]
    npp = int(round(np.sqrt(k))) // 2
    vals = gather_windows(np.asarray(y), a, b, npp)       # (R, n, k)
    phi = np.sqrt(tau2 + gamma)
    return np.einsum("rnk,nk->rn", vals, W) + phi[None, :] * xi


def box_groups(obs_xy, x0, y0, dx, dy):
    """Observations grouped by grid box: ascending index arrays, one per box
    that holds an observation, ordered by their first member."""
    obs_xy = np.asarray(obs_xy, dtype=np.float64).reshape(-1, 2)
    ix = np.floor((obs_xy[:, 0] - x0) / dx).astype(np.int64)
    iy = np.floor((obs_xy[:, 1] - y0) / dy).astype(np.int64)
    groups = {}
    for i, key in enumerate(zip(ix, iy)):
        groups.setdefault(key, []).append(i)
    return [np.array(v) for v in groups.values()]


def box_noise_factors(obs_xy, cov: Cov, x0, y0, dx, dy, a, b, W, tau2, groups, npp):
    """{first member: L_G} for every box with more than one observation:
    lower Cholesky factor of tau^2 I + Gamma_G (the conditional covariance of
    y(s_G) given the box's window plus the nugget)."""
    obs_xy = np.asarray(obs_xy, dtype=np.float64).reshape(-1, 2)
    p, q = window_offsets(npp)
    out = {}
    for G in groups:
        if len(G) < 2:
            continue
        i0 = G[0]
        gx = x0 + (a[i0] + p) * dx
        gy = y0 + (b[i0] + q) * dy
        kG = np.stack([covariance(gx - obs_xy[j, 0], gy - obs_xy[j, 1], cov) for j in G])
        S = obs_xy[G]
        KGG = covariance(S[:, 0:1] - S[None, :, 0], S[:, 1:2] - S[None, :, 1], cov)
        Gam = KGG - W[G] @ kG.T
        out[int(i0)] = np.linalg.cholesky(tau2 * np.eye(len(G)) + 0.5 * (Gam + Gam.T))
    return out


def synthetic_obs_joint(y, a, b, W, gamma, tau2, xi, groups, factors):
    """Step 3 with boxes sampled jointly: z*_G = W1_G y + L_G xi_G; boxes with
    one observation as in synthetic_obs.  y: (R, m2, m1), xi: (R, n)."""
    k = W.shape[1]
    npp = int(round(np.sqrt(k))) // 2
    vals = gather_windows(np.asarray(y), a, b, npp)
    z = np.einsum("rnk,nk->rn", vals, W)
    xi = np.asarray(xi, dtype=np.float64)
    noise = np.sqrt(tau2 + gamma)[None, :] * xi
    for G in groups:
        if len(G) > 1:
            noise[:, G] = xi[:, G] @ factors[int(G[0])].T
    return z + noise
