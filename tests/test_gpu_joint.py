"""Joint sampling of observations that share a grid box
(CESIM_PARAM_JOINT_BOXES) through the C ABI: parity with the oracle's joint
variant, the reduction to the independent sampling when every box holds one
observation, refactoring for a new nugget, and the size limit."""
import numpy as np
import pytest

from oracle import localkrige as olk
from oracle.covariance import Cov as OCov
from oracle.pipeline import Grid as OGrid
from oracle.pipeline import conditional_simulation, draw_observations
from paper_2109_11044_amd import cesim, workloads

pytestmark = pytest.mark.gpu


def rel_rms(a, b):
    a = np.asarray(a, dtype=np.float64).reshape(a.shape[0], -1)
    b = np.asarray(b, dtype=np.float64).reshape(b.shape[0], -1)
    return np.sqrt(np.mean((a - b) ** 2, axis=1) / np.mean(b ** 2, axis=1))


def run(prec, m, xy, z, cov, k, tau2s, R, joint, seed=5):
    out = []
    with cesim.Context(cesim.make_cov(*cov), cesim.unit_square_grid(m), prec) as ctx:
        ctx.set_param(cesim.PARAM_JOINT_BOXES, 1 if joint else 0)
        ctx.offgrid(xy, k)
        for tau2 in tau2s:
            f = ctx.simulate(R, seed, 1)
            ctx.condition(z, tau2, f)
            out.append(f.cpu().numpy())
        t = ctx.info()["t1"]
    return out, t


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("mixed", 1e-4)])
@pytest.mark.parametrize("cov,k", [((0.5, 1.0, 0.15), 16), ((1.5, 1.0, 0.2, 2.0, 0.5), 36)])
def test_joint_boxes_match_oracle(prec, tol, cov, k):
    m, n, R = 40, 400, 4
    xy = workloads.locations("clustered", n, seed=8)
    g = OGrid.unit_square(m)
    groups = olk.box_groups(xy, g.x0, g.y0, g.dx, g.dy)
    assert max(len(G) for G in groups) >= 3
    ocov = OCov(*cov)
    z = draw_observations(xy, ocov, 0.05, seed=0)
    got, t = run(prec, m, xy, z, cov, k, [0.05, 0.02], R, True)
    for tau2, f in zip([0.05, 0.02], got):
        ref = conditional_simulation(ocov, g, xy, z, tau2, k, 5, R, 1, t, t, joint=True)
        err = rel_rms(f, ref["v"])
        assert np.all(err < tol), (tau2, err)


def test_one_observation_per_box_is_bit_identical():
    import torch
    m = 32
    cells = np.array([[3, 4], [10, 20], [25, 7], [15, 15], [30, 30], [1, 28]])
    xy = (cells + 0.4) / (m - 1)
    z = np.linspace(-1, 1, len(xy))
    a, _ = run("fp64", m, xy, z, (0.5, 1.0, 0.2), 16, [0.05], 3, False)
    b, _ = run("fp64", m, xy, z, (0.5, 1.0, 0.2), 16, [0.05], 3, True)
    assert np.array_equal(a[0], b[0])


def test_box_size_limit():
    import torch
    xy = 0.3 + np.random.default_rng(1).uniform(0, 0.01, (40, 2))      # 40 stations, one box
    with cesim.Context(cesim.make_cov(0.5, 1.0, 0.2), cesim.unit_square_grid(16)) as ctx:
        ctx.set_param(cesim.PARAM_JOINT_BOXES, 1)
        ctx.offgrid(xy, 4)
        f = ctx.simulate(2, 1)
        with pytest.raises(cesim.CesimError) as e:
            ctx.condition(np.zeros(40), 0.05, f)
        assert e.value.name == "INVALID_ARG"
        ctx.set_param(cesim.PARAM_JOINT_BOXES, 0)
        ctx.condition(np.zeros(40), 0.05, f)                          # independent sampling
        assert torch.isfinite(f).all()
        with pytest.raises(cesim.CesimError):
            ctx.set_param(cesim.PARAM_JOINT_BOXES, 2)
