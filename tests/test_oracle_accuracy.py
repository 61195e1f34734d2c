"""Pins of the prediction standard errors (oracle/accuracy.py): SE_E
against the exact conditional covariance of eq. (4), SE_L against the
covariance of the whole simulation's linear map (Section 3.1 by an
independent route), SE_L = SE_E for observations on nodes, and a loose
statistical comparison with the fractions printed in Table 1 (Section 3.4)."""
import os

import numpy as np
import pytest

from oracle import accuracy as acc
from oracle import localkrige as lk
from oracle.covariance import Cov
from oracle.pipeline import Grid, exact_conditional, linear_map

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table1_local_kriging_sig3.txt")


@pytest.mark.parametrize("cov,tau2", [(Cov(0.5, 1.0, 0.3), 0.05), (Cov(1.5, 1.2, 0.4, 2.0, 0.6), 0.1)])
def test_se_exact_is_the_conditional_covariance(cov, tau2):
    g = Grid.unit_square(9)
    xy = np.random.default_rng(1).uniform(0, 1, (7, 2))
    _, C = exact_conditional(cov, g, xy, np.zeros(7), tau2)
    np.testing.assert_allclose(acc.se_exact(cov, g, xy, tau2) ** 2, np.diag(C), atol=1e-13)


@pytest.mark.parametrize("cov,k,tau2", [(Cov(0.5, 1.0, 0.35), 4, 0.05),
                                        (Cov(1.5, 1.0, 0.3, 2.0, 0.3), 16, 0.1),
                                        (Cov(1.0, 1.0, 0.25), 16, 0.02)])
def test_se_local_is_the_variance_of_the_simulation(cov, k, tau2):
    g = Grid.unit_square(6)
    xy = np.random.default_rng(2).uniform(0, 1, (5, 2))
    Me, Mx = linear_map(cov, g, xy, tau2, k)
    var = np.diag(Me @ Me.T + Mx @ Mx.T)
    np.testing.assert_allclose(acc.se_local(cov, g, xy, tau2, k) ** 2, var, atol=1e-12)


def test_observations_on_nodes_make_local_exact():
    g = Grid.unit_square(12)
    xy = np.array([[2, 3], [7, 9], [10, 1], [5, 5]]) / 11.0
    cov = Cov(0.5, 1.0, 0.2)
    np.testing.assert_allclose(acc.se_local(cov, g, xy, 0.05, 16), acc.se_exact(cov, g, xy, 0.05),
                               atol=1e-12)


def test_listed_nodes_equal_the_full_grid():
    g = Grid(10, 7, 0.2, -0.1, 0.11, 0.13)
    xy = np.random.default_rng(5).uniform(0, 1, (9, 2))
    cov = Cov(1.0, 1.1, 0.3)
    rows = np.array([69, 0, 33, 34, 5])
    np.testing.assert_allclose(acc.se_exact(cov, g, xy, 0.05, rows),
                               acc.se_exact(cov, g, xy, 0.05)[rows], atol=1e-14)
    np.testing.assert_allclose(acc.se_local(cov, g, xy, 0.05, 16, rows),
                               acc.se_local(cov, g, xy, 0.05, 16)[rows], atol=1e-13)


def test_table1_fractions_loosely():
    """Exponential covariance, 61 x 61 grid on [0, 60]^2, 35 uniform
    observations, tau = 0.1: mean over 8 configurations of the fraction of
    nodes correct to three significant figures, within 0.12 of the printed
    means for n_p = 1, 2, 3 (the windows here are clamped at the grid edge
    where the paper pads the grid, which lowers the fractions), and
    increasing in n_p."""
    rows = np.loadtxt(GOLDEN)
    g = Grid(61, 61, 0.0, 0.0, 1.0, 1.0)
    rng = np.random.default_rng(0)
    for th in (6.68, 23.37):
        row = rows[(rows[:, 0] == th) & (rows[:, 1] == 0.1)][0]
        cov = Cov(0.5, 1.0, th)
        fr = {k: [] for k in (4, 16, 36)}
        for _ in range(8):
            xy = rng.uniform(0, 60, (35, 2))
            e = acc.se_exact(cov, g, xy, 0.01)
            for k in fr:
                fr[k].append(acc.fraction_sig3(acc.se_local(cov, g, xy, 0.01, k), e))
        means = [np.mean(fr[k]) for k in (4, 16, 36)]
        assert means[0] < means[1] < means[2]
        for got, paper in zip(means, row[[2, 4, 6]]):
            assert abs(got - paper) < 0.12, (th, got, paper)


def test_study_ranges_give_five_percent_and_table1_thetas():
    """The study's ranges (Section 3.3): the correlation is 5 % at 20, 45
    and 70 units for both smoothness values, and for the exponential they
    round to the ranges printed in Table 1."""
    from paper_2109_11044_amd import workloads
    from oracle.covariance import cross_covariance
    for c in workloads.study_cases():
        cov = Cov(c["nu"], 1.0, c["theta"])
        r = cross_covariance(np.array([[0.0, 0.0]]), np.array([[c["distance"], 0.0]]), cov)
        assert abs(r[0, 0] - 0.05) < 1e-12, c
    printed = sorted(set(np.loadtxt(GOLDEN)[:, 0]))
    got = [round(workloads.study_range(0.5, d), 2) for d in workloads.STUDY_DISTANCES]
    assert got == printed
    assert len(workloads.study_cases()) == 18


def test_three_significant_figures_against_decimal_formatting():
    """round_sig against Python's correctly rounded decimal formatting
    (values drawn away from rounding ties), and fraction_sig3 on a hand
    example."""
    x = np.random.default_rng(8).uniform(0.05, 3.0, 2000)
    ref = np.array([float(f"{v:.2e}") for v in x])
    assert np.allclose(acc.round_sig(x), ref, rtol=1e-14, atol=0)
    np.testing.assert_array_equal(acc.round_sig(np.array([0.123449, 0.98765, 12.3449, 0.00012351])),
                                  np.array([0.123, 0.988, 12.3, 0.000124]))
    assert acc.fraction_sig3(np.array([0.5004, 0.5006, 1.2345]),
                             np.array([0.5001, 0.5001, 1.2351])) == pytest.approx(1.0 / 3.0)


def test_padded_grid_centres_every_window():
    """Section 2.1 widens the grid by at least n_p grid units: on the study
    grid widened by n_p on every side no window is clamped, every one is the
    2 n_p x 2 n_p block of nodes around its observation's box (brute force),
    and on the original nodes SE_E is unchanged (it does not involve the
    grid) while SE_L changes only where clamping moved windows."""
    from paper_2109_11044_amd import workloads
    rng = np.random.default_rng(5)
    xy = rng.uniform(0, 60, (35, 2))
    xy[0] = (60.0, 60.0)                       # corner of the domain
    xy[1] = (0.0, 37.5)                        # left edge
    xy[2] = (59.7, 30.2)                       # one box from the right edge
    cov = Cov(0.5, 1.0, 15.02)
    for npp in (1, 2, 3):
        k = (2 * npp) ** 2
        gp = Grid(*workloads.study_grid(npp))
        a, b = lk.window_corners(xy, gp.x0, gp.y0, gp.dx, gp.dy, gp.m1, gp.m2, npp)
        for i, (x, y) in enumerate(xy):
            # nodes with |x - node| < n_p per axis, counted from the node at floor(x)
            bx, by = int(np.floor(x)), int(np.floor(y))
            assert a[i] == (bx - npp + 1) - int(gp.x0) and b[i] == (by - npp + 1) - int(gp.y0)
        rows = np.array([(j + npp) * gp.m1 + i + npp for j in range(61) for i in range(61)])
        g0 = Grid(61, 61, 0.0, 0.0, 1.0, 1.0)
        e0 = acc.se_exact(cov, g0, xy, 0.01)
        np.testing.assert_allclose(acc.se_exact(cov, gp, xy, 0.01)[rows], e0, rtol=1e-13)
        lp = acc.se_local(cov, gp, xy, 0.01, k)[rows]
        l0 = acc.se_local(cov, g0, xy, 0.01, k)
        a0, b0 = lk.window_corners(xy, 0.0, 0.0, 1.0, 1.0, 61, 61, npp)
        moved = np.any(a0 != a - npp) or np.any(b0 != b - npp)
        # n_p = 1 windows are the box corners, which the 61 x 61 grid holds
        # (a station exactly on the last grid line sits on a node, where the
        # moved window gives the same weights); from n_p = 2 the stations
        # near the edge were clamped before and SE_L changes
        assert moved
        assert np.all(lp > 0) and (np.allclose(lp, l0, rtol=1e-12) == (npp == 1))
