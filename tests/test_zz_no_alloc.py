"""The allocation-free draw entry point, ce_simulate_noalloc, through the C
ABI: its fields equal those of ce_simulate bit for bit on two calls in a
row, the second with a smaller input, on both precisions and on the
register-FFT and general paths; a pair buffer larger than the static array
is refused."""
import ctypes

import pytest

from paper_2109_11044_amd import cesim

pytestmark = pytest.mark.gpu


def noalloc(ctx, nreal, seed, first, out):
    return cesim.lib().ce_simulate_noalloc(ctx._h, int(nreal), int(seed), int(first),
                                           ctypes.c_void_p(out.data_ptr()))


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
@pytest.mark.parametrize("grid", [
    cesim.unit_square_grid(1024),                       # 2048 torus: several chunks of pairs
    cesim.Grid(40, 24, 0.0, 0.0, 0.02, 0.03, 0, 0),     # rectangular: general FFT path
])
def test_noalloc_equals_simulate(prec, grid):
    import torch
    print(f"noalloc vs simulate: {prec} {grid.m1}x{grid.m2}", flush=True)
    with cesim.Context(cesim.make_cov(0.5, 1.0, 0.05), grid, prec) as ctx:
        for nreal, seed, first in ((13, 7, 3), (5, 2, 0)):      # second call smaller
            ref = ctx.simulate(nreal, seed, first)
            out = torch.full_like(ref, float("nan"))
            assert noalloc(ctx, nreal, seed, first, out) == 0
            torch.cuda.synchronize()
            assert torch.equal(out, ref), (nreal, first)
        # the conditioning step accepts the batch it drew
        xy = torch.rand((20, 2), dtype=torch.float64).numpy() * 0.55 + 0.05   # inside both grids
        ctx.offgrid(xy, 4)
        f = torch.empty_like(ref)
        assert noalloc(ctx, 5, 2, 0, f) == 0
        ctx.condition(xy[:, 0] * 0.0, 0.1, f)
        assert bool(torch.isfinite(f).all())


def test_noalloc_refuses_pairs_beyond_the_array():
    import torch
    # FP64 on a 4096 torus: one pair needs 16 * 4096 * 2048 B = 128 MiB > 64 MiB
    with cesim.Context(cesim.make_cov(0.5, 1.0, 0.02), cesim.unit_square_grid(2048),
                       "fp64") as ctx:
        out = torch.empty((1, 2048, 2048), dtype=torch.float64, device="cuda")
        assert noalloc(ctx, 1, 1, 0, out) == 1            # INVALID_ARG
    assert cesim.lib().ce_simulate_noalloc(None, 1, 1, 0, None) == 1
