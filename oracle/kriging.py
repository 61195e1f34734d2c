"""Kriging from the observations onto the grid (oracle side; test
infrastructure only).

Section 2 lists the conditional simulation steps: (1) the prediction y_hat on
the grid from the data z, (4) the prediction y_tilde from the synthetic data
z*, (5) v = y_hat + (y(S^g) - y_tilde).  Both predictions are the simple
Kriging mean of eq. (4), Section 3,

    E[y(S^g) | z] = K12 (K22 + tau^2 I)^{-1} z,

with K12[g, i] = C(g - s_i) and K22[i, j] = C(s_i - s_j); item (d) of
Section 2.1 keeps the plain nugget tau^2 here.  Written with one Cholesky
factor of A = K22 + tau^2 I:

    c_hat = A^{-1} z,   alpha*_r = A^{-1} z*_r,
    v_r   = y_r + K12 (c_hat - alpha*_r).

K12 is never stored: it is evaluated in chunks of grid rows.

Pins (tests/test_oracle_pipeline.py): with tau^2 = 0 and observations on
nodes the conditional fields reproduce the data exactly; with all
observations on nodes the covariance of the pipeline's linear map equals the
conditional covariance of eq. (4); in general it equals the closed form of
Section 3.1.
"""

import numpy as np
from scipy.linalg import cho_factor, cho_solve

from .covariance import Cov, cross_covariance


def obs_matrix(obs_xy, cov: Cov, tau2):
    """A = K22 + tau^2 I."""
    obs_xy = np.asarray(obs_xy, dtype=np.float64).reshape(-1, 2)
    A = cross_covariance(obs_xy, obs_xy, cov)
    A[np.diag_indices_from(A)] += tau2
    return A


class NotPositiveDefinite(ValueError):
    pass


def factor(obs_xy, cov: Cov, tau2):
    try:
        return cho_factor(obs_matrix(obs_xy, cov, tau2), lower=True)
    except np.linalg.LinAlgError as e:
        raise NotPositiveDefinite(str(e))


def coefficients(fac, z, zstar):
    """B[:, r] = A^{-1} (z - z*_r); z (n,), zstar (R, n) -> (n, R)."""
    rhs = np.asarray(z, dtype=np.float64)[:, None] - np.asarray(zstar).T
    return cho_solve(fac, rhs)


def grid_points(x0, y0, dx, dy, m1, m2, rows=None):
    """Grid node coordinates (x fastest) of the given grid rows j."""
    rows = np.arange(m2) if rows is None else np.asarray(rows)
    i = np.arange(m1)
    gx = np.broadcast_to(x0 + i[None, :] * dx, (rows.size, m1))
    gy = np.broadcast_to(y0 + rows[:, None] * dy, (rows.size, m1))
    return np.stack([gx.reshape(-1), gy.reshape(-1)], axis=1)


def krige_to_grid(B, obs_xy, cov: Cov, x0, y0, dx, dy, m1, m2, rows=None,
                  chunk_rows=16):
    """K12 B for the given grid rows: (R, len(rows), m1)."""
    rows = np.arange(m2) if rows is None else np.asarray(rows)
    R = B.shape[1]
    out = np.empty((R, rows.size, m1))
    for s in range(0, rows.size, chunk_rows):
        rr = rows[s:s + chunk_rows]
        K12 = cross_covariance(grid_points(x0, y0, dx, dy, m1, m2, rr),
                               obs_xy, cov)
        out[:, s:s + rr.size, :] = (K12 @ B).T.reshape(R, rr.size, m1)
    return out


def condition_fields(y, B, obs_xy, cov: Cov, x0, y0, dx, dy, m1, m2):
    """Step 5: v_r = y_r + K12 B[:, r]."""
    return np.asarray(y) + krige_to_grid(B, obs_xy, cov, x0, y0, dx, dy,
                                         m1, m2)
