"""Pins of the joint sampling of observations that share a grid box
(oracle/localkrige.py, Section 2.1 and Section 3.6): the block factors
against the Schur complement of the joint covariance, the reduction to the
independent sampling for boxes with one observation, and the exact
conditional law (eq. (4)) when all observations lie in one box whose window
is the whole grid -- which the independent sampling does not reach."""
import numpy as np
import pytest

from oracle import localkrige as lk
from oracle.covariance import Cov, cross_covariance
from oracle.pipeline import Grid, exact_conditional, linear_map, offgrid_setup


def test_box_factor_is_the_conditional_covariance():
    g = Grid.unit_square(16)
    cov = Cov(1.0, 1.3, 0.2, 1.5, 0.4)
    rng = np.random.default_rng(3)
    box = np.array([5, 9]) / 15.0
    xy = box + rng.uniform(0, 1.0 / 15.0, (4, 2))
    xy = np.vstack([xy, [[0.9, 0.1]]])
    a, b, W, gamma = offgrid_setup(xy, cov, g, 16)
    groups = lk.box_groups(xy, g.x0, g.y0, g.dx, g.dy)
    assert sorted(len(G) for G in groups) == [1, 4]
    fac = lk.box_noise_factors(xy, cov, g.x0, g.y0, g.dx, g.dy, a, b, W, 0.07, groups, 2)
    L = fac[0]
    p, q = lk.window_offsets(2)
    nodes = np.stack([g.x0 + (a[0] + p) * g.dx, g.y0 + (b[0] + q) * g.dy], axis=1)
    Knn = cross_covariance(nodes, nodes, cov)
    Kng = cross_covariance(nodes, xy[:4], cov)
    Kgg = cross_covariance(xy[:4], xy[:4], cov)
    schur = Kgg - Kng.T @ np.linalg.solve(Knn, Kng)
    np.testing.assert_allclose(L @ L.T, schur + 0.07 * np.eye(4), atol=1e-12)
    np.testing.assert_allclose(np.diag(schur), gamma[:4], atol=1e-12)


def test_one_observation_per_box_matches_independent_sampling():
    g = Grid.unit_square(12)
    cov = Cov(0.5, 1.0, 0.2)
    xy = (np.array([[1, 2], [4, 7], [9, 3], [6, 6]]) + 0.37) / 11.0
    a, b, W, gamma = offgrid_setup(xy, cov, g, 16)
    groups = lk.box_groups(xy, g.x0, g.y0, g.dx, g.dy)
    rng = np.random.default_rng(0)
    y = rng.standard_normal((3, 12, 12))
    xi = rng.standard_normal((3, 4))
    fac = lk.box_noise_factors(xy, cov, g.x0, g.y0, g.dx, g.dy, a, b, W, 0.05, groups, 2)
    assert fac == {}
    np.testing.assert_array_equal(lk.synthetic_obs_joint(y, a, b, W, gamma, 0.05, xi, groups, fac),
                                  lk.synthetic_obs(y, a, b, W, gamma, 0.05, xi))


@pytest.mark.parametrize("cov", [Cov(1.5, 1.0, 0.5), Cov(0.5, 1.0, 0.4, 2.0, 0.7)])
def test_one_box_full_grid_window_is_exact_only_when_joint(cov):
    g = Grid.unit_square(4)
    xy = np.array([[0.41, 0.47], [0.52, 0.61], [0.63, 0.39]])    # all in box (1, 1)
    tau2 = 0.05
    _, C = exact_conditional(cov, g, xy, np.zeros(3), tau2)
    Me, Mx = linear_map(cov, g, xy, tau2, 16, joint=True)       # 2 n_p = m
    assert np.max(np.abs(Me @ Me.T + Mx @ Mx.T - C)) < 1e-12
    Me, Mx = linear_map(cov, g, xy, tau2, 16, joint=False)
    assert np.max(np.abs(Me @ Me.T + Mx @ Mx.T - C)) > 1e-4
