"""Batches of uneven events through the C ABI: parity with the oracle per
event, bit-equality with the one-event path, replays with a realization
offset, and per-event error statuses."""
import numpy as np
import pytest

from oracle.covariance import Cov as OCov
from oracle.pipeline import Grid as OGrid
from oracle.pipeline import conditional_simulation, draw_observations
from paper_2109_11044_amd import cesim, workloads

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-10
MIXED_TOL = 1e-4


def rel_rms(a, b):
    a = np.asarray(a, dtype=np.float64).reshape(a.shape[0], -1)
    b = np.asarray(b, dtype=np.float64).reshape(b.shape[0], -1)
    return np.sqrt(np.mean((a - b) ** 2, axis=1) / np.mean(b ** 2, axis=1))


# (m1, m2, nu, range, ratio, angle, n, locs, k, tau2, nreal, first, seed, id)
SMALL_EVENTS = [
    (32, 32, 0.5, 0.1, 1.0, 0.0, 40, "uniform", 16, 0.05, 5, 0, 11, 3),
    (48, 48, 1.5, 0.15, 2.0, 0.6, 150, "clustered", 36, 0.1, 4, 0, 12, 0),
    (40, 24, 1.0, 0.1, 1.0, 0.0, 90, "uniform", 4, 0.02, 3, 2, 13, 7),
    (64, 64, 0.5, 0.05, 1.5, 1.1, 200, "clustered", 16, 0.05, 7, 5, 14, 1),
    (24, 24, 0.5, 0.2, 1.0, 0.0, 10, "uniform", 64, 0.03, 2, 0, 15, 2),
]


def make_events(spec=SMALL_EVENTS):
    evs, orc = [], []
    for e, (m1, m2, nu, th, ra, an, n, locs, k, tau2, R, first, seed, eid) in enumerate(spec):
        dx = 1.0 / (m1 - 1)
        grid = cesim.Grid(m1, m2, 0.0, 0.0, dx, dx, 0, 0)
        ogrid = OGrid(m1, m2, 0.0, 0.0, dx, dx)
        xy = workloads.locations(locs, n, seed=100 + e)
        xy[:, 1] *= (m2 - 1) * dx            # stations inside a rectangular grid
        ocov = OCov(nu, 1.0, th, ra, an)
        z = draw_observations(xy, ocov, tau2, seed=0)
        evs.append(dict(cov=cesim.make_cov(nu, 1.0, th, ra, an), grid=grid, obs_xy=xy, z=z,
                        nugget=tau2, k=k, nreal=R, first_real=first, seed=seed, event_id=eid))
        orc.append(dict(cov=ocov, grid=ogrid))
    return evs, orc


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_batch_matches_oracle(prec):
    evs, orc = make_events()
    print(f"batch of {len(evs)} events, {prec}", flush=True)
    with cesim.Batch(evs, prec) as b:
        fields = [f.cpu().numpy() for f in b.run(0)]
        tori = [b.info(e)["t1"] for e in range(len(evs))], [b.info(e)["t2"] for e in range(len(evs))]
    tol = FP64_TOL if prec == "fp64" else MIXED_TOL
    for e, (ev, o) in enumerate(zip(evs, orc)):
        ref = conditional_simulation(o["cov"], o["grid"], ev["obs_xy"], ev["z"], ev["nugget"],
                                     ev["k"], ev["seed"], ev["nreal"], ev["first_real"],
                                     tori[0][e], tori[1][e], event=ev["event_id"])
        err = rel_rms(fields[e], ref["v"])
        assert np.all(err < tol), (e, err)


def single_event(ev, prec, offset=0):
    with cesim.Context(ev["cov"], ev["grid"], prec) as ctx:
        ctx.set_param(cesim.PARAM_EVENT_ID, ev["event_id"])
        ctx.offgrid(ev["obs_xy"], ev["k"])
        f = ctx.simulate(ev["nreal"], ev["seed"], ev["first_real"] + offset)
        ctx.condition(ev["z"], ev["nugget"], f)
        return f.cpu()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_batch_bit_equal_to_single_event_path_and_replays(prec):
    import torch
    evs, _ = make_events()
    with cesim.Batch(evs, prec) as b:
        first = [f.cpu() for f in b.run(0)]
        later = [f.cpu() for f in b.run(9)]
        again = [f.cpu() for f in b.run(0)]
    for e, ev in enumerate(evs):
        assert torch.equal(first[e], single_event(ev, prec)), e
        assert torch.equal(later[e], single_event(ev, prec, 9)), e
        assert torch.equal(again[e], first[e]), e
        assert not torch.equal(later[e], first[e]), e


def test_event_id_changes_the_draw():
    import torch
    evs, _ = make_events(SMALL_EVENTS[:1])
    a = single_event(evs[0], "fp64")
    evs[0]["event_id"] += 1
    b = single_event(evs[0], "fp64")
    assert not torch.equal(a, b)


def test_batch_error_statuses():
    evs, _ = make_events(SMALL_EVENTS[:3])
    bad = dict(evs[1])
    bad["nreal"] = 0
    with pytest.raises(cesim.BatchError) as ei:
        cesim.Batch([evs[0], bad, evs[2]], "fp64")
    assert ei.value.name == "INVALID_ARG"
    assert ei.value.event_status == ["OK", "INVALID_ARG", "OK"]
    # forced torus with negative eigenvalues (Matern 3/2, range 0.3, 32^2 on 64^2)
    neg = dict(evs[0], cov=cesim.make_cov(1.5, 1.0, 0.3), grid=cesim.unit_square_grid(32, 64))
    with pytest.raises(cesim.BatchError) as ei:
        cesim.Batch([evs[0], neg], "mixed")
    assert ei.value.event_status[1] == "NEGATIVE_EIGENVALUE"
    # two stations at one point without nugget: K22 singular
    xy = evs[2]["obs_xy"].copy()
    xy[1] = xy[0]
    sing = dict(evs[2], obs_xy=xy, nugget=0.0)
    with pytest.raises(cesim.BatchError) as ei:
        cesim.Batch([evs[0], sing, evs[1]], "fp64")
    assert ei.value.name == "NOT_POSITIVE_DEFINITE"
    assert ei.value.event_status == ["OK", "NOT_POSITIVE_DEFINITE", "OK"]
    # the library is still usable
    with cesim.Batch(evs, "fp64") as b:
        assert all(np.isfinite(f.cpu().numpy()).all() for f in b.run(0))
