"""The blocked factorization of K22 + tau^2 I (64-column diagonal blocks,
trailing updates split between the next block column and the rest) and the
256-block substitutions, at station counts around every block boundary:
the coefficients alpha_r = A^{-1}(z - z*_r) and the conditional fields of the
FP64 path against the oracle (Section 2, steps 4 and 5), and the status of a
system that is not positive definite at each position of its failing pivot
relative to the blocks."""
import numpy as np
import pytest

from oracle.covariance import Cov as OCov
from oracle.pipeline import Grid as OGrid
from oracle.pipeline import conditional_simulation, draw_observations
from paper_2109_11044_amd import cesim, workloads

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n", [1, 2, 63, 64, 65, 127, 128, 129, 192, 193, 255, 256, 257, 321])
def test_coefficients_and_fields_at_block_boundaries(n):
    cov, m, k, tau2, R, seed = (1.0, 1.0, 0.1), 24, 16, 0.03, 3, 4
    xy = workloads.locations("uniform", n, seed=100 + n)
    oc = OCov(*cov)
    z = draw_observations(xy, oc, tau2, seed=1)
    print(f"factor blocks: n={n}", flush=True)
    with cesim.Context(cesim.make_cov(*cov), cesim.unit_square_grid(m), "fp64") as ctx:
        ctx.offgrid(xy, k)
        f = ctx.simulate(R, seed)
        ctx.condition(z, tau2, f)
        t = ctx.info()["t1"]
        got_v = f.cpu().numpy()
        got_a = ctx.coefficients().cpu().numpy()
    ref = conditional_simulation(oc, OGrid.unit_square(m), xy, z, tau2, k, seed, R, 0, t, t)
    ea = np.max(np.abs(got_a - ref["B"].T)) / np.abs(ref["B"]).max()
    ev = np.max(np.abs(got_v - ref["v"])) / np.abs(ref["v"]).max()
    assert ea < 1e-9 and ev < 1e-10, (ea, ev)


@pytest.mark.parametrize("dup", [0, 62, 63, 64, 130])
def test_failing_pivot_in_any_block(dup):
    """140 stations on a lattice of spacing 1/12 with an exponential range of
    1e-4: every correlation between distinct stations underflows to exactly
    0, so with nugget 0 the system is the identity except that station
    dup + 1 repeats station dup.  The pivot of row dup + 1 is then exactly
    0, in the first block, at a block's last or first row, or in a later
    block; condition() reports NOT_POSITIVE_DEFINITE and leaves the fields
    unchanged."""
    import torch
    n = 140
    g = (np.arange(12) + 0.5) / 12
    xy = np.stack(np.meshgrid(g, g, indexing="xy"), axis=-1).reshape(-1, 2)[:n].copy()
    xy[dup + 1] = xy[dup]
    print(f"failing pivot: row {dup + 1}", flush=True)
    with cesim.Context(cesim.make_cov(0.5, 1.0, 1e-4), cesim.unit_square_grid(20), "fp64") as ctx:
        ctx.offgrid(xy, 4)
        f = ctx.simulate(2, 3)
        before = f.clone()
        with pytest.raises(cesim.CesimError) as e:
            ctx.condition(np.zeros(n), 0.0, f)
        assert e.value.name == "NOT_POSITIVE_DEFINITE"
        torch.cuda.synchronize()
        assert torch.equal(f, before)
