"""Pins of the oracle's local Kriging (Section 2.1, Section 3.1,
Section 3.6)."""
import numpy as np
import pytest

from oracle import localkrige as lk
from oracle.covariance import Cov, cross_covariance, covariance
from oracle.pipeline import Grid, offgrid_setup


def test_observation_on_node_gives_indicator():
    g = Grid.unit_square(20)
    cov = Cov(0.5, 1.0, 0.2)
    nodes = np.array([[5, 7], [0, 0], [19, 19], [10, 3]])
    xy = np.stack([g.x0 + nodes[:, 0] * g.dx, g.y0 + nodes[:, 1] * g.dy], 1)
    for k in (4, 16, 36):
        npp = int(np.sqrt(k)) // 2
        a, b, W, gamma = offgrid_setup(xy, cov, g, k)
        p, q = lk.window_offsets(npp)
        for i in range(len(xy)):
            e = ((a[i] + p == nodes[i, 0]) & (b[i] + q == nodes[i, 1])).astype(float)
            assert e.sum() == 1
            assert np.max(np.abs(W[i] - e)) < 1e-12
            assert gamma[i] < 1e-12


def test_window_is_the_nearest_nodes_per_axis():
    g = Grid(40, 30, 0.5, -1.0, 0.25, 0.2)
    rng = np.random.default_rng(3)
    for npp in (1, 2, 3, 4):
        # interior points: the window holds exactly the 2 n_p nodes closest to s
        xy = np.stack([rng.uniform(g.x0 + npp * g.dx, g.x0 + (g.m1 - 1 - npp) * g.dx, 200),
                       rng.uniform(g.y0 + npp * g.dy, g.y0 + (g.m2 - 1 - npp) * g.dy, 200)], 1)
        a, b = lk.window_corners(xy, g.x0, g.y0, g.dx, g.dy, g.m1, g.m2, npp)
        for i in range(200):
            dxs = np.abs(g.x0 + np.arange(g.m1) * g.dx - xy[i, 0])
            dys = np.abs(g.y0 + np.arange(g.m2) * g.dy - xy[i, 1])
            assert set(np.argsort(dxs, kind="stable")[:2 * npp]) == set(range(a[i], a[i] + 2 * npp))
            assert set(np.argsort(dys, kind="stable")[:2 * npp]) == set(range(b[i], b[i] + 2 * npp))
    # edges: the window stays inside the grid with full size
    edge = np.array([[g.x0, g.y0], [g.x0 + (g.m1 - 1) * g.dx, g.y0 + (g.m2 - 1) * g.dy],
                     [g.x0 + 0.3 * g.dx, g.y0 + (g.m2 - 1.5) * g.dy]])
    a, b = lk.window_corners(edge, g.x0, g.y0, g.dx, g.dy, g.m1, g.m2, 3)
    assert list(a) == [0, g.m1 - 6, 0] and list(b) == [0, g.m2 - 6, g.m2 - 6]


def test_weights_and_gamma_match_schur_complement():
    """w and gamma from the inverse of the joint covariance of
    (window, s): gamma = 1 / P_ss and w = -P_ws / P_ss."""
    g = Grid.unit_square(25)
    rng = np.random.default_rng(8)
    xy = rng.uniform(0, 1, (25, 2))
    for cov, k in [(Cov(0.5, 1.0, 0.1), 16), (Cov(1.5, 2.0, 0.15, 2.0, 0.4), 36),
                   (Cov(1.0, 1.0, 0.2), 4)]:
        npp = int(np.sqrt(k)) // 2
        a, b, W, gamma = offgrid_setup(xy, cov, g, k)
        p, q = lk.window_offsets(npp)
        for i in range(len(xy)):
            pts = np.stack([g.x0 + (a[i] + p) * g.dx, g.y0 + (b[i] + q) * g.dy], 1)
            allp = np.vstack([pts, xy[i:i + 1]])
            P = np.linalg.inv(cross_covariance(allp, allp, cov))
            gam = 1.0 / P[k, k]
            w = -P[:k, k] / P[k, k]
            assert gamma[i] == pytest.approx(gam, rel=1e-8, abs=1e-13)
            assert np.max(np.abs(W[i] - w)) < 1e-8 * max(1.0, np.abs(w).max())


def test_gamma_decreases_with_neighbourhood_order():
    g = Grid.unit_square(40)
    cov = Cov(1.5, 1.0, 0.1)
    rng = np.random.default_rng(4)
    xy = rng.uniform(0.3, 0.7, (50, 2))       # interior: windows are nested
    prev = None
    for k in (4, 16, 36, 64):
        _, _, _, gamma = offgrid_setup(xy, cov, g, k)
        assert np.all(gamma >= 0) and np.all(gamma <= cov.sigma2)
        if prev is not None:
            assert np.all(gamma <= prev + 1e-15)
        prev = gamma


def test_invalid_k_rejected():
    g = Grid.unit_square(10)
    with pytest.raises(ValueError):
        offgrid_setup(np.array([[0.5, 0.5]]), Cov(), g, 15)
    with pytest.raises(ValueError):
        offgrid_setup(np.array([[0.5, 0.5]]), Cov(), g, 144)


def test_synthetic_obs_is_weights_plus_scaled_noise():
    g = Grid.unit_square(12)
    cov = Cov(0.5, 1.0, 0.2)
    xy = np.array([[0.31, 0.52], [0.9, 0.1]])
    a, b, W, gamma = offgrid_setup(xy, cov, g, 16)
    y = np.arange(144.0).reshape(1, 12, 12)
    xi = np.array([[0.5, -2.0]])
    zs = lk.synthetic_obs(y, a, b, W, gamma, 0.3, xi)
    p, q = lk.window_offsets(2)
    for i in range(2):
        vals = y[0, b[i] + q, a[i] + p]
        assert zs[0, i] == pytest.approx(vals @ W[i] + np.sqrt(0.3 + gamma[i]) * xi[0, i],
                                         rel=1e-14)
