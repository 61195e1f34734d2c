"""GPU parity of the HIP path against the oracle (through the C ABI)."""
import numpy as np
import pytest

from oracle import ce as oce
from oracle.covariance import Cov as OCov
from oracle.pipeline import Grid as OGrid
from oracle.pipeline import (conditional_simulation, draw_observations,
                             offgrid_setup, setup)
from paper_2109_11044_amd import cesim, workloads

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-10       # relative RMS per field, plain FP64 path
MIXED_TOL = 1e-4       # relative RMS per field, mixed path


def rel_rms(a, b):
    a = np.asarray(a, dtype=np.float64).reshape(a.shape[0], -1)
    b = np.asarray(b, dtype=np.float64).reshape(b.shape[0], -1)
    return np.sqrt(np.mean((a - b) ** 2, axis=1) / np.mean(b ** 2, axis=1))


def ctx_for(nu, sigma2, rng_, m, prec="fp64", torus=0, aniso=(1.0, 0.0)):
    return cesim.Context(cesim.make_cov(nu, sigma2, rng_, *aniso),
                         cesim.unit_square_grid(m, torus), prec)


@pytest.mark.parametrize("nu,theta,m,torus,aniso", [
    (0.5, 0.1, 64, 128, (1.0, 0.0)),       # exponential, 64^2 grid, 128 torus
    (1.5, 0.2, 24, 0, (1.0, 0.0)),          # ladder, radix-3 sizes
    (1.0, 0.15, 40, 0, (2.0, 0.6)),         # Bessel K1, anisotropic
    (0.5, 0.05, 30, 75, (1.5, 1.1)),        # odd torus (radix 3 and 5)
])
def test_spectrum_matches_oracle(nu, theta, m, torus, aniso):
    with ctx_for(nu, 1.0, theta, m, "fp64", torus, aniso) as ctx:
        info = ctx.info()
        s = ctx.spectrum().cpu().numpy()
    t1, t2, sref, oinfo = setup(OCov(nu, 1.0, theta, *aniso), OGrid.unit_square(m),
                                torus or None, torus or None)
    assert (info["t1"], info["t2"]) == (t1, t2)
    N = t1 * t2
    assert np.max(np.abs(s * np.sqrt(N) - sref)) < 1e-12 * sref.max()
    assert info["lam_min"] == pytest.approx(oinfo["lam_min"], abs=1e-11 * oinfo["lam_max"])
    assert info["lam_sum"] == pytest.approx(N * 1.0, rel=1e-10)
    # the setup's acceptance checks: real spectrum and the trace identity
    assert info["max_imag"] <= 1e-12 * info["lam_max"]
    assert info["max_imag"] == pytest.approx(oinfo["max_imag"], abs=1e-13 * oinfo["lam_max"])


def test_ladder_moves_past_negative_torus():
    """nu = 1, theta = 0.15, m = 256: 512 is rejected, 768 accepted."""
    with ctx_for(1.0, 1.0, 0.15, 256) as ctx:
        info = ctx.info()
    assert (info["t1"], info["t2"]) == (768, 768) and info["torus_tries"] == 2


@pytest.mark.parametrize("prec,tol", [("fp64", FP64_TOL), ("mixed", MIXED_TOL)])
@pytest.mark.parametrize("m,torus,nreal,first", [
    (64, 128, 5, 0), (24, 0, 3, 7), (30, 75, 4, 1),          # small, radix 3 and 5
    (128, 256, 3, 0), (512, 1024, 2, 5),                     # power-of-two register path
    (1024, 2048, 3, 997),                                    # full-size torus of the benchmark
    (128, 384, 3, 0), (256, 768, 2, 1), (512, 1536, 3, 2),   # 3 * 2^a: FP32 register path
    (1024, 3072, 1, 0), (1024, 6144, 1, 4),
])
def test_unconditional_draw_matches_oracle(prec, tol, m, torus, nreal, first):
    cov = (0.5, 1.0, 0.1)
    with ctx_for(*cov, m, prec, torus) as ctx:
        f = ctx.simulate(nreal, seed=2, first_real=first).cpu().numpy()
        t1, t2 = ctx.info()["t1"], ctx.info()["t2"]
    _, _, sref, _ = setup(OCov(*cov), OGrid.unit_square(m), t1, t2)
    ref = oce.ce_draw(sref, 2, range(first, first + nreal), m, m)
    err = rel_rms(f, ref)
    assert np.all(err < tol), err


def test_rectangular_grid_draw():
    """m1 != m2 (different torus sizes per axis) through the general path."""
    cov = OCov(1.5, 1.0, 0.12, 2.0, 0.3)
    g = cesim.Grid(40, 24, 0.0, 0.0, 0.02, 0.03, 0, 0)
    with cesim.Context(cesim.make_cov(1.5, 1.0, 0.12, 2.0, 0.3), g, "fp64") as ctx:
        f = ctx.simulate(3, seed=4).cpu().numpy()
        t1, t2 = ctx.info()["t1"], ctx.info()["t2"]
    og = OGrid(40, 24, 0.0, 0.0, 0.02, 0.03)
    _, _, sref, _ = setup(cov, og, t1, t2)
    ref = oce.ce_draw(sref, 4, range(3), 40, 24)
    assert np.all(rel_rms(f, ref) < FP64_TOL)


def test_draw_independent_of_batching():
    with ctx_for(0.5, 1.0, 0.1, 48, "fp64") as ctx:
        a = ctx.simulate(7, seed=11).cpu().numpy()
        b = ctx.simulate(3, seed=11, first_real=4).cpu().numpy()
    assert np.array_equal(a[4:], b)


@pytest.mark.parametrize("k", [4, 16, 36, 64])
def test_local_kriging_weights_match_oracle(k):
    m = 50
    xy = workloads.clustered_locations(300, seed=5)
    xy[:4] = [[0.0, 0.0], [1.0, 1.0], [0.5, 0.5], [1.0, 0.0]]
    xy[4] = [10 / 49, 20 / 49]                      # on a node
    cov = (1.5, 1.0, 0.1)
    with ctx_for(*cov, m, "fp64") as ctx:
        ctx.offgrid(xy, k)
        cor, w, gm = (t.cpu().numpy() for t in ctx.weights())
    a, b, W, gamma = offgrid_setup(xy, OCov(*cov), OGrid.unit_square(m), k)
    assert np.array_equal(cor[:, 0], a) and np.array_equal(cor[:, 1], b)
    assert np.max(np.abs(w - W)) < 1e-9 * max(1.0, np.abs(W).max())
    assert np.max(np.abs(gm - gamma)) < 1e-12


def run_both(wl, prec, nreal, seed=2, first=0, torus=0):
    xy = wl.obs_xy()
    ocov = OCov(wl.nu, wl.sigma2, wl.range, wl.aniso_ratio, wl.aniso_angle)
    z = draw_observations(xy, ocov, wl.tau2, seed=0)
    with cesim.Context(cesim.make_cov(wl.nu, wl.sigma2, wl.range, wl.aniso_ratio,
                                      wl.aniso_angle),
                       cesim.unit_square_grid(wl.m, torus or wl.torus), prec) as ctx:
        ctx.offgrid(xy, wl.k)
        f = ctx.simulate(nreal, seed, first)
        ctx.condition(z, wl.tau2, f)
        v = f.cpu().numpy()
        t1 = ctx.info()["t1"]
        B = ctx.coefficients().cpu().numpy()
    ref = conditional_simulation(ocov, OGrid.unit_square(wl.m), xy, z, wl.tau2, wl.k,
                                 seed, nreal, first, t1, t1)
    return v, B, ref


def test_conditional_fp64_small_exact_config():
    v, B, ref = run_both(workloads.C1, "fp64", workloads.C1.nreal)
    assert np.max(np.abs(B - ref["B"].T)) < 1e-9 * np.abs(ref["B"]).max()
    err = rel_rms(v, ref["v"])
    assert np.all(err < FP64_TOL), err


def test_conditional_mixed_small_exact_config():
    v, B, ref = run_both(workloads.C1, "mixed", workloads.C1.nreal)
    err = rel_rms(v, ref["v"])
    assert np.all(err < MIXED_TOL), err


def test_mixed_new_observations_rerun_the_prediction():
    """Two conditionings on one mixed context with different observed values:
    each runs its own prediction of the data term, whose workgroups take
    their items from a counter reset before every launch, and each matches
    the oracle (eq. (4) with the new values)."""
    wl = workloads.C1
    xy = wl.obs_xy()
    ocov = OCov(wl.nu, wl.sigma2, wl.range, wl.aniso_ratio, wl.aniso_angle)
    seed, nreal = 2, wl.nreal
    with cesim.Context(cesim.make_cov(wl.nu, wl.sigma2, wl.range, wl.aniso_ratio,
                                      wl.aniso_angle),
                       cesim.unit_square_grid(wl.m, wl.torus), "mixed") as ctx:
        ctx.offgrid(xy, wl.k)
        for zseed in (0, 1):
            z = draw_observations(xy, ocov, wl.tau2, seed=zseed)
            f = ctx.simulate(nreal, seed, 0)
            ctx.condition(z, wl.tau2, f)
            v = f.cpu().numpy()
            t1 = ctx.info()["t1"]
            ref = conditional_simulation(ocov, OGrid.unit_square(wl.m), xy, z, wl.tau2, wl.k,
                                         seed, nreal, 0, t1, t1)
            err = rel_rms(v, ref["v"])
            assert np.all(err < MIXED_TOL), (zseed, err)
