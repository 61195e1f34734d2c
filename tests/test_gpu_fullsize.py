"""Full-size workloads on the GPU, checked against the oracle on sampled
outputs (realizations and grid nodes the oracle computes one by one):
the 64-event batch in the launch configuration the benchmark times, the
512^2 Matern nu = 1 workload with 2000 clustered stations, and the
ShakeMap-scale 2048^2 workload with 20000 clustered stations streamed in
batches of 64 realizations."""
import numpy as np
import pytest

from oracle import ce as oce
from oracle import kriging, localkrige, philox
from oracle.covariance import Cov as OCov
from oracle.covariance import cross_covariance
from oracle.pipeline import Grid as OGrid
from oracle.pipeline import offgrid_setup, setup
from paper_2109_11044_amd import cesim, workloads

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-10
MIXED_TOL = 1e-4


def rel_rms(a, b):
    return np.sqrt(np.mean((a - b) ** 2, axis=1) / np.mean(b ** 2, axis=1))


def sampled_reference(ocov, m, xy, z, tau2, k, reals, t, nodes, seed, event=0, fac=None):
    """Oracle v_r at sampled nodes of an m x m unit-square grid for the
    realizations ``reals`` (steps 1-5 of Section 2; Section 2.1 (a)-(d))."""
    g = OGrid.unit_square(m)
    _, _, s, _ = setup(ocov, g, t, t)
    y = oce.ce_draw(s, seed, reals, m, m, event)
    a, b, W, gamma = offgrid_setup(xy, ocov, g, k)
    xi = philox.offgrid_noise(seed, len(xy), reals, event)
    zs = localkrige.synthetic_obs(y, a, b, W, gamma, tau2, xi)
    if fac is None:
        fac = kriging.factor(xy, ocov, tau2)
    B = kriging.coefficients(fac, z, zs)
    K12 = cross_covariance(g.points()[nodes], xy, ocov)
    return y.reshape(len(reals), -1)[:, nodes] + (K12 @ B).T


def test_batch_of_64_uneven_events_sampled():
    """The benchmark's 64-event table (grids 128^2-512^2, tori up to 4096,
    100-3000 stations, 200 realizations each) run as one batch in mixed
    precision; five events of different grid and torus sizes compared on
    two realizations at 2048 sampled nodes each."""
    import torch
    table = workloads.event_table(64)
    inp = workloads.event_inputs(table)
    seed = 2
    evs = [dict(cov=cesim.make_cov(d["nu"], d["sigma2"], d["range"], d["aniso_ratio"],
                                   d["aniso_angle"]),
                grid=cesim.unit_square_grid(d["m"]), obs_xy=d["obs_xy"], z=d["z"],
                nugget=d["nugget"], k=d["k"], nreal=d["nreal"], first_real=0, seed=seed,
                event_id=d["event_id"]) for d in inp]
    print("planning 64 events", flush=True)
    with cesim.Batch(evs, "mixed") as b:
        fields = b.run(0)
        tori = [b.info(e)["t1"] for e in range(64)]
        # smallest grid, a 3 * 2^a torus, a Matern 3/2 event, the largest torus
        pick = {int(np.argmin([d["m"] for d in inp]))}
        pick.add(next(e for e, t in enumerate(tori) if t % 3 == 0 and inp[e]["m"] == 256))
        pick.add(next(e for e, d in enumerate(inp) if d["nu"] == 1.5 and d["m"] == 512))
        pick.add(int(np.argmax(tori)))
        pick.add(next(e for e, t in enumerate(tori) if t % 3 == 0 and inp[e]["m"] == 512))
        reals = [0, 199]
        rng = np.random.default_rng(5)
        got = {}
        for e in sorted(pick):
            m = inp[e]["m"]
            nodes = rng.choice(m * m, 2048, replace=False)
            got[e] = (nodes, fields[e].view(200, -1)[reals][:, torch.as_tensor(
                nodes, device="cuda")].cpu().numpy())
    for e, (nodes, g) in got.items():
        d = inp[e]
        print(f"event {e}: m {d['m']} torus {tori[e]} n {len(d['z'])} nu {d['nu']}", flush=True)
        ocov = OCov(d["nu"], d["sigma2"], d["range"], d["aniso_ratio"], d["aniso_angle"])
        ref = sampled_reference(ocov, d["m"], d["obs_xy"], d["z"], d["nugget"], d["k"], reals,
                                tori[e], nodes, seed, event=e)
        err = rel_rms(g.astype(np.float64), ref)
        assert np.all(err < MIXED_TOL), (e, err)


@pytest.mark.parametrize("prec,tol", [("mixed", MIXED_TOL), ("fp64", FP64_TOL)])
def test_matern1_512_clustered_sampled(prec, tol):
    """512^2 grid, Matern nu = 1, range 0.1, nugget 0.05, 2000 clustered
    stations, 6x6 windows, 200 realizations in one call; realizations 3 and
    150 at 2048 sampled nodes."""
    import torch
    wl = workloads.C4
    xy = wl.obs_xy()
    ocov = OCov(wl.nu, wl.sigma2, wl.range)
    z = workloads.iid_values(wl.n, wl.sigma2 + wl.tau2)
    dt = torch.float64 if prec == "fp64" else torch.float32
    with cesim.Context(cesim.make_cov(wl.nu, wl.sigma2, wl.range),
                       cesim.unit_square_grid(wl.m), prec) as ctx:
        ctx.offgrid(xy, wl.k)
        f = torch.empty((wl.nreal, wl.m, wl.m), dtype=dt, device="cuda")
        ctx.simulate(wl.nreal, 7, out=f)
        ctx.condition(z, wl.tau2, f)
        t = ctx.info()["t1"]
        reals = [3, 150]
        nodes = np.random.default_rng(6).choice(wl.m * wl.m, 2048, replace=False)
        got = f.view(wl.nreal, -1)[reals][:, torch.as_tensor(nodes, device="cuda")]
        got = got.cpu().numpy().astype(np.float64)
    ref = sampled_reference(ocov, wl.m, xy, z, wl.tau2, wl.k, reals, t, nodes, 7)
    assert np.all(rel_rms(got, ref) < tol)


@pytest.fixture(scope="module")
def shakemap_factor():
    wl = workloads.C5
    xy = wl.obs_xy()
    ocov = OCov(wl.nu, wl.sigma2, wl.range)
    print("oracle Cholesky of the 20000-station system", flush=True)
    return xy, ocov, kriging.factor(xy, ocov, wl.tau2)


@pytest.mark.parametrize("prec,tol", [("mixed", MIXED_TOL), ("fp64", FP64_TOL)])
def test_shakemap_scale_streamed_batches_sampled(prec, tol, shakemap_factor):
    """2048^2 grid on a 4096^2 torus, exponential range 0.02, nugget 0.02,
    20000 clustered stations, 6x6 windows; realizations streamed in batches
    of 64 through one context (the factorisation is reused); realization 5
    of the first batch and 100 of the second compared at 2048 sampled
    nodes."""
    import torch
    wl = workloads.C5
    xy, ocov, fac = shakemap_factor
    z = workloads.iid_values(wl.n, wl.sigma2 + wl.tau2)
    dt = torch.float64 if prec == "fp64" else torch.float32
    nodes = np.random.default_rng(8).choice(wl.m * wl.m, 2048, replace=False)
    idx = torch.as_tensor(nodes, device="cuda")
    got = []
    with cesim.Context(cesim.make_cov(wl.nu, wl.sigma2, wl.range),
                       cesim.unit_square_grid(wl.m), prec) as ctx:
        ctx.offgrid(xy, wl.k)
        f = torch.empty((wl.batch, wl.m, wl.m), dtype=dt, device="cuda")
        for first, r in ((0, 5), (64, 100)):
            print(f"{prec}: batch at {first}", flush=True)
            ctx.simulate(wl.batch, 9, first, out=f)
            ctx.condition(z, wl.tau2, f)
            got.append(f[r - first].view(-1)[idx].cpu().numpy().astype(np.float64))
        t = ctx.info()["t1"]
        del f
    assert t == 4096
    ref = sampled_reference(ocov, wl.m, xy, z, wl.tau2, wl.k, [5, 100], t, nodes, 9, fac=fac)
    assert np.all(rel_rms(np.stack(got), ref) < tol)


@pytest.mark.parametrize("split", [0, 1, 2])
def test_shakemap_scale_split_errors_sampled(split, shakemap_factor):
    """The ShakeMap-scale configuration's cross-covariance product in each
    arithmetic of the mixed path (FP16 or BF16 three-product split, plain
    FP32): realizations 0 and 1 at 2048 sampled nodes against the oracle;
    the error is printed for the record."""
    import torch
    wl = workloads.C5
    xy, ocov, fac = shakemap_factor
    z = workloads.iid_values(wl.n, wl.sigma2 + wl.tau2)
    nodes = np.random.default_rng(10).choice(wl.m * wl.m, 2048, replace=False)
    with cesim.Context(cesim.make_cov(wl.nu, wl.sigma2, wl.range),
                       cesim.unit_square_grid(wl.m), "mixed") as ctx:
        ctx.set_param(cesim.PARAM_GEMM_SPLIT, split)
        ctx.offgrid(xy, wl.k)
        f = torch.empty((2, wl.m, wl.m), dtype=torch.float32, device="cuda")
        ctx.simulate(2, 11, 0, out=f)
        ctx.condition(z, wl.tau2, f)
        got = f.view(2, -1)[:, torch.as_tensor(nodes, device="cuda")].cpu().numpy()
        t = ctx.info()["t1"]
        del f
    ref = sampled_reference(ocov, wl.m, xy, z, wl.tau2, wl.k, [0, 1], t, nodes, 11, fac=fac)
    err = rel_rms(got.astype(np.float64), ref)
    print(f"\nsplit-error C5 split={split}: max {err.max():.3e}", flush=True)
    assert np.all(err < MIXED_TOL), err
