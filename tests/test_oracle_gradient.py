"""Pins of the oracle's reference adjoint (oracle/gradient.py): the
theta-derivative of the Matern correlation, the mean-noise form of the
linear ensemble statistic, and every gradient component against central
finite differences (h = 1e-6, FP64, common random numbers) of the ensemble
statistic of the full simulation."""
import numpy as np
import pytest

from oracle import gradient
from oracle.covariance import Cov, covariance
from oracle.pipeline import Grid, draw_observations
from paper_2109_11044_amd import workloads


@pytest.mark.parametrize("nu", [0.5, 1.5])
def test_closed_forms_of_g_match_the_bessel_form(nu):
    x = np.concatenate([np.linspace(1e-6, 0.1, 50), np.linspace(0.1, 30.0, 300)])
    np.testing.assert_allclose(gradient.matern_g(x, nu), gradient.matern_g_bessel(x, nu),
                               rtol=1e-12, atol=1e-300)


@pytest.mark.parametrize("nu", [0.5, 1.0, 1.5])
@pytest.mark.parametrize("ratio,angle", [(1.0, 0.0), (2.5, 0.7)])
def test_dcov_is_the_theta_derivative(nu, ratio, angle):
    rng = np.random.default_rng(1)
    hx, hy = rng.uniform(-0.5, 0.5, 200), rng.uniform(-0.5, 0.5, 200)
    th, h = 0.17, 1e-6
    cp = covariance(hx, hy, Cov(nu, 1.3, th + h, ratio, angle))
    cm = covariance(hx, hy, Cov(nu, 1.3, th - h, ratio, angle))
    fd = (cp - cm) / (2 * h)
    np.testing.assert_allclose(gradient.dcov_dtheta(hx, hy, Cov(nu, 1.3, th, ratio, angle)), fd,
                               rtol=1e-7, atol=1e-9)


def small_case(nu=1.0, ratio=1.0, angle=0.0):
    m, t = 16, 32
    grid = Grid.unit_square(m)
    xy = workloads.uniform_locations(12, seed=4)
    cov = Cov(nu, 1.0, 0.15, ratio, angle)
    tau2 = 0.1
    z = draw_observations(xy, cov, tau2, seed=0)
    w = np.random.default_rng(9).standard_normal((m, m))
    return dict(grid=grid, obs_xy=xy, z=z, tau2=tau2, k=16, seed=5, nreal=3, weights=w,
                t1=t, t2=t), cov


def test_mean_noise_statistic_equals_ensemble_statistic():
    kw, cov = small_case(1.5, 2.0, 0.4)
    g = gradient.linear_stat_gradient(cov, **kw)
    L = gradient.ensemble_stat(cov, **kw)
    assert abs(g["L"] - L) <= 1e-11 * max(1.0, abs(L))


@pytest.mark.parametrize("nu,ratio,angle", [(0.5, 1.0, 0.0), (1.0, 1.0, 0.0), (1.5, 1.0, 0.0),
                                            (1.0, 2.0, 0.9)])
def test_gradient_matches_central_differences(nu, ratio, angle):
    kw, cov = small_case(nu, ratio, angle)
    g = gradient.linear_stat_gradient(cov, **kw)
    h = 1e-6

    def L(cv=cov, **over):
        args = dict(kw)
        args.update(over)
        return gradient.ensemble_stat(cv, **args)

    def close(adj, fd):
        assert abs(adj - fd) <= 1e-6 * max(abs(fd), 1e-3), (adj, fd)

    close(g["d_range"], (L(Cov(nu, 1.0, 0.15 + h, ratio, angle))
                         - L(Cov(nu, 1.0, 0.15 - h, ratio, angle))) / (2 * h))
    close(g["d_sigma2"], (L(Cov(nu, 1.0 + h, 0.15, ratio, angle))
                          - L(Cov(nu, 1.0 - h, 0.15, ratio, angle))) / (2 * h))
    close(g["d_tau2"], (L(tau2=kw["tau2"] + h) - L(tau2=kw["tau2"] - h)) / (2 * h))
    for i in (0, 7):
        zp, zm = kw["z"].copy(), kw["z"].copy()
        zp[i] += h
        zm[i] -= h
        close(g["d_z"][i], (L(z=zp) - L(z=zm)) / (2 * h))


def nonlinear_stat(cov, grid, obs_xy, z, tau2, k, seed, nreal, weights, t1, t2,
                   which="variance"):
    """From the full simulation: S = sum_g w_g Var_r(v_r[g]) (population
    variance over the ensemble; dS/dv_r = (2/R) w (v_r - mean)), or the
    second moment S = sum_g w_g mean_r v_r[g]^2 (dS/dv_r = (2/R) w v_r)."""
    from oracle.pipeline import conditional_simulation
    v = conditional_simulation(cov, grid, obs_xy, z, tau2, k, seed, nreal, 0, t1, t2)["v"]
    w = np.asarray(weights).reshape(grid.m2, grid.m1)
    if which == "variance":
        mean = v.mean(axis=0)
        return float(np.sum(w * v.var(axis=0))), (2.0 / nreal) * w[None] * (v - mean[None])
    return float(np.sum(w * np.mean(v * v, axis=0))), (2.0 / nreal) * w[None] * v


@pytest.mark.parametrize("nu,ratio,angle,which", [(0.5, 1.0, 0.0, "variance"),
                                                  (1.0, 2.0, 0.9, "variance"),
                                                  (1.5, 1.0, 0.0, "moment2")])
def test_fields_vjp_gives_nonlinear_statistic_gradients(nu, ratio, angle, which):
    """The gradient of a non-linear ensemble statistic (the weighted sum of
    the per-node ensemble variances, or of the second moments) by the
    fields' vector-Jacobian product against central differences of the
    statistic from the full simulation."""
    kw, cov = small_case(nu, ratio, angle)
    args = {key: kw[key] for key in ("grid", "obs_xy", "z", "tau2", "k", "seed", "nreal",
                                     "weights", "t1", "t2")}
    args["which"] = which
    S0, vbar = nonlinear_stat(cov, **args)
    kvjp = {key: args[key] for key in ("grid", "obs_xy", "z", "tau2", "k", "seed", "t1", "t2")}
    g = gradient.fields_vjp(cov, vbar=vbar, **kvjp)
    h = 1e-6

    def S(cv=cov, **over):
        a = dict(args)
        a.update(over)
        return nonlinear_stat(cv, **a)[0]

    def close(adj, fd):
        # central differences carry about eps |S| / h of rounding
        assert abs(adj - fd) <= 1e-6 * abs(fd) + 1e-8 * abs(S0), (adj, fd)

    close(g["d_range"], (S(Cov(nu, 1.0, 0.15 + h, ratio, angle))
                         - S(Cov(nu, 1.0, 0.15 - h, ratio, angle))) / (2 * h))
    close(g["d_sigma2"], (S(Cov(nu, 1.0 + h, 0.15, ratio, angle))
                          - S(Cov(nu, 1.0 - h, 0.15, ratio, angle))) / (2 * h))
    close(g["d_tau2"], (S(tau2=args["tau2"] + h) - S(tau2=args["tau2"] - h)) / (2 * h))
    for i in (0, 7):
        zp, zm = args["z"].copy(), args["z"].copy()
        zp[i] += h
        zm[i] -= h
        close(g["d_z"][i], (S(z=zp) - S(z=zm)) / (2 * h))
    if which == "variance":
        # z moves every realization by the same prediction, so the ensemble
        # variance does not depend on it
        assert np.max(np.abs(g["d_z"])) < 1e-10 * abs(S0)
