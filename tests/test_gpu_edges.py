"""Edge cases of the conditional simulation through the C ABI, against the
oracle: one station and one realization, zero nugget with stations on grid
nodes (the fields reproduce the data there), an odd realization count with
a station count one past a 64-block, stations on the far grid edges, more
stations than grid cells, and realization counters next to the top of the
index range."""
import numpy as np
import pytest

from oracle.covariance import Cov as OCov
from oracle.pipeline import Grid as OGrid
from oracle.pipeline import conditional_simulation, draw_observations
from paper_2109_11044_amd import cesim, workloads

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "mixed": 1e-4}


def rel_rms(a, b):
    a = np.asarray(a, dtype=np.float64).reshape(a.shape[0], -1)
    b = np.asarray(b, dtype=np.float64).reshape(b.shape[0], -1)
    return np.sqrt(np.mean((a - b) ** 2, axis=1) / np.mean(b ** 2, axis=1))


def run(prec, m, xy, z, cov, tau2, k, R, seed=3, first=0, torus=0):
    with cesim.Context(cesim.make_cov(*cov), cesim.unit_square_grid(m, torus), prec) as ctx:
        ctx.offgrid(xy, k)
        f = ctx.simulate(R, seed, first)
        ctx.condition(z, tau2, f)
        t = ctx.info()["t1"]
        return f.cpu().numpy(), t


def check(prec, m, xy, z, cov, tau2, k, R, seed=3, first=0, torus=0, tol=None):
    got, t = run(prec, m, xy, z, cov, tau2, k, R, seed, first, torus)
    ref = conditional_simulation(OCov(*cov), OGrid.unit_square(m), xy, z, tau2, k, seed, R, first,
                                 t, t)
    err = rel_rms(got, ref["v"])
    assert np.all(err < (tol or TOL[prec])), err
    return got


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_one_station_one_realization(prec):
    xy = np.array([[0.37, 0.61]])
    check(prec, 32, xy, np.array([0.8]), (1.0, 1.0, 0.2), 0.05, 16, 1)


def test_zero_nugget_reproduces_data_on_nodes():
    """A station on a node has gamma = 0 in exact arithmetic; each code rounds
    it to O(k eps sigma^2) and, with zero nugget, phi = sqrt(gamma) turns
    that into O(sqrt(k eps)) ~ 1e-7: at the station v = z - phi xi, and the
    two FP64 codes agree to that level, not to 1e-10."""
    m = 33
    nodes = np.array([[4, 7], [20, 3], [11, 29], [31, 16], [17, 17]])
    xy = nodes / (m - 1.0)
    z = np.array([1.5, -0.7, 0.2, 2.1, -1.3])
    bound = np.sqrt(16 * np.finfo(float).eps)          # phi at most sqrt(k eps sigma^2)
    got = check("fp64", m, xy, z, (0.5, 1.0, 0.15), 0.0, 16, 3, tol=4 * bound)
    at = got[:, nodes[:, 1], nodes[:, 0]]
    assert np.max(np.abs(at - z[None, :])) < 5 * bound


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_odd_realizations_and_ragged_station_count(prec):
    xy = workloads.locations("clustered", 65, seed=12)
    cov = (1.0, 1.0, 0.12)
    z = draw_observations(xy, OCov(*cov), 0.04, seed=0)
    check(prec, 48, xy, z, cov, 0.04, 36, 7)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_stations_on_the_far_edges(prec):
    xy = np.array([[1.0, 1.0], [1.0, 0.3], [0.45, 1.0], [0.0, 1.0], [1.0, 0.0], [0.0, 0.0],
                   [0.999999, 0.5]])
    cov = (1.5, 1.0, 0.2, 2.0, 0.3)
    z = draw_observations(xy, OCov(*cov), 0.05, seed=0)
    check(prec, 40, xy, z, cov, 0.05, 64, 3)


def test_more_stations_than_grid_cells():
    xy = workloads.locations("uniform", 700, seed=5)
    cov = (0.5, 1.0, 0.3)
    z = draw_observations(xy, OCov(*cov), 0.1, seed=0)
    check("fp64", 24, xy, z, cov, 0.1, 64, 2)


def test_realization_counters_at_the_top_of_the_range():
    xy = workloads.locations("uniform", 30, seed=9)
    cov = (0.5, 1.0, 0.1)
    z = draw_observations(xy, OCov(*cov), 0.05, seed=0)
    check("fp64", 32, xy, z, cov, 0.05, 16, 4, seed=2**40 + 17, first=2**31 - 5)
