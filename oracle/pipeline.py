"""The five-step conditional simulation with local Kriging, end to end, plus
test-only outputs (oracle side; test infrastructure only).

Section 2 gives the algorithm (steps 1-5) and Section 2.1 items (a)-(d) the
local-Kriging approximation of steps 2-4:

  (a) y_r on the grid by circulant embedding           -> ce.ce_draw
  (b)+(c) z*_r = W1 y_r + sqrt(tau^2 + gamma) xi_r      -> localkrige
  (1),(4),(5) v_r = y_r + K12 A^{-1} (z - z*_r)         -> kriging
  (d) the grid prediction uses tau^2 alone.

Random inputs: eps_r from Philox stream 0 and xi_r from stream 1, both keyed
by the seed, the absolute realization index r and the event index; the CE
draw of realization r uses the torus noise of both members of its pair
(eps_{2P}, eps_{2P+1}, P = r // 2).

Test-only helpers build, for tiny problems, the explicit linear map of the
pipeline from (eps_{2P}, eps_{2P+1}, xi) to v - y_hat, the paper's
closed-form covariance of that map (Section 3.1) and the exact conditional
law (eq. (4), Section 3).
"""

from dataclasses import dataclass

import numpy as np

from . import ce, kriging, localkrige, philox
from .covariance import Cov, cross_covariance


@dataclass(frozen=True)
class Grid:
    m1: int
    m2: int
    x0: float = 0.0
    y0: float = 0.0
    dx: float = 1.0
    dy: float = 1.0

    @staticmethod
    def unit_square(m):
        """m x m nodes on [0, 1]^2 including both edges: spacing 1/(m-1)."""
        return Grid(m, m, 0.0, 0.0, 1.0 / (m - 1), 1.0 / (m - 1))

    def points(self):
        return kriging.grid_points(self.x0, self.y0, self.dx, self.dy,
                                   self.m1, self.m2)


def setup(cov: Cov, grid: Grid, t1=None, t2=None):
    return ce.ce_setup(cov, grid.dx, grid.dy, grid.m1, grid.m2, t1, t2)


def offgrid_setup(obs_xy, cov: Cov, grid: Grid, k):
    return localkrige.local_krige(obs_xy, cov, grid.x0, grid.y0, grid.dx,
                                  grid.dy, grid.m1, grid.m2, k)


def draw_observations(obs_xy, cov: Cov, tau2, seed=0):
    """Observed values drawn from the model: z = L22 xi + tau xi', with
    L22 the Cholesky factor of K22 and xi, xi' from Philox stream 2
    (realizations 0 and 1, event 0)."""
    obs_xy = np.asarray(obs_xy, dtype=np.float64).reshape(-1, 2)
    n = obs_xy.shape[0]
    K22 = cross_covariance(obs_xy, obs_xy, cov)
    L = np.linalg.cholesky(K22 + 1e-12 * cov.sigma2 * np.eye(n))
    xi = philox.normals(seed, n, 0, 0, philox.STREAM_FIXTURE)
    xi2 = philox.normals(seed, n, 1, 0, philox.STREAM_FIXTURE)
    return L @ xi + np.sqrt(tau2) * xi2


def synthetic(y, obs_xy, cov: Cov, grid: Grid, a, b, W, gamma, tau2, xi, joint):
    """Step 3 with the local Kriging of Section 2.1, each observation on its
    own (joint=False) or boxes of several observations jointly."""
    if not joint:
        return localkrige.synthetic_obs(y, a, b, W, gamma, tau2, xi)
    npp = int(round(np.sqrt(W.shape[1]))) // 2
    groups = localkrige.box_groups(obs_xy, grid.x0, grid.y0, grid.dx, grid.dy)
    fac = localkrige.box_noise_factors(obs_xy, cov, grid.x0, grid.y0, grid.dx, grid.dy, a, b,
                                       W, tau2, groups, npp)
    return localkrige.synthetic_obs_joint(y, a, b, W, gamma, tau2, xi, groups, fac)


def conditional_simulation(cov: Cov, grid: Grid, obs_xy, z, tau2, k, seed,
                           nreal, first_real=0, t1=None, t2=None, event=0, joint=False):
    """Run steps 1-5 for realizations first_real .. first_real + nreal - 1
    (noise counters carry ``event`` in their third word; joint: boxes of
    several observations sampled jointly).

    Returns a dict of every intermediate: torus, sqrt_lam, y, window
    corners a/b, W, gamma, xi, zstar, B, v."""
    t1, t2, s, info = setup(cov, grid, t1, t2)
    reals = np.arange(first_real, first_real + nreal)
    y = ce.ce_draw(s, seed, reals, grid.m1, grid.m2, event)
    a, b, W, gamma = offgrid_setup(obs_xy, cov, grid, k)
    xi = philox.offgrid_noise(seed, len(obs_xy), reals, event)
    zstar = synthetic(y, obs_xy, cov, grid, a, b, W, gamma, tau2, xi, joint)
    fac = kriging.factor(obs_xy, cov, tau2)
    B = kriging.coefficients(fac, z, zstar)
    v = kriging.condition_fields(y, B, obs_xy, cov, grid.x0, grid.y0,
                                 grid.dx, grid.dy, grid.m1, grid.m2)
    return dict(t1=t1, t2=t2, info=info, sqrt_lam=s, y=y, a=a, b=b,
                W=W, gamma=gamma, xi=xi, zstar=zstar, B=B, v=v)


# ---------------------------------------------------------------- test only

def draw_matrix(sqrt_lam, m1, m2, part=0):
    """Explicit matrix (M, 2N) of the CE draw of one member of a pair, from
    the pair's noise [eps_{2P}; eps_{2P+1}] (each T2*T1) to y (m2*m1):
    part 0 is realization 2P (Re W), part 1 realization 2P + 1 (Im W)."""
    t2, t1 = sqrt_lam.shape
    N = t1 * t2
    cols = []
    for half in (0, 1):
        for q in range(N):
            e = np.zeros(N)
            e[q] = 1.0
            z = np.zeros(N)
            pair = (e, z) if half == 0 else (z, e)
            f = ce.ce_draw_pair(sqrt_lam, pair[0].reshape(t2, t1), pair[1].reshape(t2, t1), m1, m2)
            cols.append(f[part].reshape(-1))
    return np.stack(cols, axis=1)


def linear_map(cov: Cov, grid: Grid, obs_xy, tau2, k, t1=None, t2=None, joint=False):
    """Matrices (Me, Mx) with v - y_hat = Me [eps_{2P}; eps_{2P+1}] + Mx xi
    for the whole pipeline, realization 2P of a pair (z enters only y_hat;
    realization 2P + 1 has the same covariance).  Tiny problems only."""
    t1, t2, s, _ = setup(cov, grid, t1, t2)
    Bce = draw_matrix(s, grid.m1, grid.m2)                  # (M, 2N)
    a, b, W, gamma = offgrid_setup(obs_xy, cov, grid, k)
    n = len(obs_xy)
    fac = kriging.factor(obs_xy, cov, tau2)
    z0 = np.zeros(n)
    # columns for eps
    Y = Bce.T.reshape(-1, grid.m2, grid.m1)                 # (2N, m2, m1)
    zs = synthetic(Y, obs_xy, cov, grid, a, b, W, gamma, tau2, np.zeros((Y.shape[0], n)),
                   joint)
    Bc = kriging.coefficients(fac, z0, zs)
    Ve = kriging.condition_fields(Y, Bc, obs_xy, cov, grid.x0, grid.y0,
                                  grid.dx, grid.dy, grid.m1, grid.m2)
    Me = Ve.reshape(Y.shape[0], -1).T
    # columns for xi
    Y0 = np.zeros((n, grid.m2, grid.m1))
    zs = synthetic(Y0, obs_xy, cov, grid, a, b, W, gamma, tau2, np.eye(n), joint)
    Bx = kriging.coefficients(fac, z0, zs)
    Vx = kriging.condition_fields(Y0, Bx, obs_xy, cov, grid.x0, grid.y0,
                                  grid.dx, grid.dy, grid.m1, grid.m2)
    Mx = Vx.reshape(n, -1).T
    return Me, Mx


def prediction(cov: Cov, grid: Grid, obs_xy, z, tau2):
    """y_hat = K12 A^{-1} z on the grid (flattened, x fastest)."""
    fac = kriging.factor(obs_xy, cov, tau2)
    c = kriging.coefficients(fac, z, np.zeros((1, len(z))))
    return kriging.krige_to_grid(c, obs_xy, cov, grid.x0, grid.y0, grid.dx,
                                 grid.dy, grid.m1, grid.m2).reshape(-1)


def exact_conditional(cov: Cov, grid: Grid, obs_xy, z, tau2):
    """Mean and covariance of y(S^g) | z from eq. (4), Section 3."""
    G = grid.points()
    K11 = cross_covariance(G, G, cov)
    K12 = cross_covariance(G, obs_xy, cov)
    A = kriging.obs_matrix(obs_xy, cov, tau2)
    mean = K12 @ np.linalg.solve(A, z)
    covm = K11 - K12 @ np.linalg.solve(A, K12.T)
    return mean, covm
