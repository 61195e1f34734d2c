"""Pins of the oracle pipeline (Section 2 steps 1-5 with Section 2.1) against
the exact conditional law (eq. (4), Section 3), the closed-form covariance of
Section 3.1, data reproduction and Monte Carlo moments."""
import numpy as np
import pytest

from oracle import kriging
from oracle import localkrige as lk
from oracle.covariance import Cov, cross_covariance
from oracle.pipeline import (Grid, conditional_simulation, draw_observations,
                             exact_conditional, linear_map, offgrid_setup,
                             prediction)


def on_node_obs(g, nodes):
    nodes = np.asarray(nodes)
    return np.stack([g.x0 + nodes[:, 0] * g.dx, g.y0 + nodes[:, 1] * g.dy], 1)


def test_zero_nugget_reproduces_data_on_nodes():
    g = Grid.unit_square(16)
    cov = Cov(0.5, 1.0, 0.25)
    xy = on_node_obs(g, [[3, 4], [10, 12], [15, 0], [7, 7]])
    z = np.array([1.0, -0.5, 2.0, 0.3])
    out = conditional_simulation(cov, g, xy, z, 0.0, 16, seed=5, nreal=3)
    for i, (ix, jy) in enumerate([[3, 4], [10, 12], [15, 0], [7, 7]]):
        # gamma is zero only up to rounding (~1e-16); its square root enters
        # the synthetic datum, so the residual is bounded by sqrt(gamma)|xi|.
        bound = 1e-10 + np.sqrt(out["gamma"][i]) * np.abs(out["xi"][:, i])
        assert np.all(np.abs(out["v"][:, jy, ix] - z[i]) <= bound)


def test_observations_on_nodes_give_exact_conditional_law():
    g = Grid.unit_square(6)
    cov = Cov(0.5, 1.0, 0.4)
    xy = on_node_obs(g, [[1, 1], [4, 2], [2, 5]])
    tau2 = 0.1
    Me, Mx = linear_map(cov, g, xy, tau2, 4)
    z = np.array([0.7, -0.2, 1.1])
    mean, C = exact_conditional(cov, g, xy, z, tau2)
    assert np.max(np.abs(Me @ Me.T + Mx @ Mx.T - C)) < 1e-12
    assert np.max(np.abs(prediction(cov, g, xy, z, tau2) - mean)) < 1e-12


def test_single_observation_full_grid_window_is_exact():
    g = Grid.unit_square(4)
    cov = Cov(1.5, 1.0, 0.5)
    xy = np.array([[0.41, 0.77]])
    tau2 = 0.05
    Me, Mx = linear_map(cov, g, xy, tau2, 16)       # 2 n_p = m
    _, C = exact_conditional(cov, g, xy, np.zeros(1), tau2)
    assert np.max(np.abs(Me @ Me.T + Mx @ Mx.T - C)) < 1e-12


def dense_w1(g, xy, a, b, W, k):
    npp = int(np.sqrt(k)) // 2
    p, q = lk.window_offsets(npp)
    W1 = np.zeros((len(xy), g.m1 * g.m2))
    for i in range(len(xy)):
        W1[i, (b[i] + q) * g.m1 + a[i] + p] = W[i]
    return W1


@pytest.mark.parametrize("cov,k,tau2", [(Cov(0.5, 1.0, 0.35), 4, 0.05),
                                        (Cov(1.5, 1.0, 0.3, 2.0, 0.3), 16, 0.1)])
def test_covariance_matches_section_3_1_closed_form(cov, k, tau2):
    g = Grid.unit_square(7)
    rng = np.random.default_rng(2)
    xy = rng.uniform(0, 1, (5, 2))
    Me, Mx = linear_map(cov, g, xy, tau2, k)
    a, b, W, gamma = offgrid_setup(xy, cov, g, k)
    G = g.points()
    K11 = cross_covariance(G, G, cov)
    K12 = cross_covariance(G, xy, cov)
    W2 = K12 @ np.linalg.inv(kriging.obs_matrix(xy, cov, tau2))
    Lam = W2 @ dense_w1(g, xy, a, b, W, k)
    I = np.eye(G.shape[0])
    closed = (Lam - I) @ K11 @ (Lam - I).T + W2 @ np.diag(tau2 + gamma) @ W2.T
    assert np.max(np.abs(Me @ Me.T + Mx @ Mx.T - closed)) < 1e-12


def test_conditional_moments_monte_carlo():
    g = Grid.unit_square(8)
    cov = Cov(0.5, 1.0, 0.3)
    rng = np.random.default_rng(6)
    xy = rng.uniform(0, 1, (6, 2))
    tau2 = 0.05
    z = draw_observations(xy, cov, tau2, seed=0)
    R = 1500
    out = conditional_simulation(cov, g, xy, z, tau2, 4, seed=9, nreal=R)
    v = out["v"].reshape(R, -1)
    yhat = prediction(cov, g, xy, z, tau2)
    Me, Mx = linear_map(cov, g, xy, tau2, 4)
    var = np.diag(Me @ Me.T + Mx @ Mx.T)
    zmean = (v.mean(0) - yhat) / np.sqrt(var / R)
    zvar = (v.var(0) - var) / (var * np.sqrt(2.0 / R))
    assert np.max(np.abs(zmean)) < 4.5 and np.max(np.abs(zvar)) < 4.5


def test_results_do_not_depend_on_batching():
    g = Grid.unit_square(10)
    cov = Cov(0.5, 1.0, 0.2)
    rng = np.random.default_rng(1)
    xy = rng.uniform(0, 1, (7, 2))
    z = draw_observations(xy, cov, 0.1)
    full = conditional_simulation(cov, g, xy, z, 0.1, 16, seed=3, nreal=5)
    part = conditional_simulation(cov, g, xy, z, 0.1, 16, seed=3, nreal=2, first_real=3)
    assert np.array_equal(full["v"][3:], part["v"])
