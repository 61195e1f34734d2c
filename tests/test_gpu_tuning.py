"""Launch shapes and autotuning on the GPU: every tile shape of the draw
passes and of the grid GEMM gives bit-identical results, and tuned contexts
and batches reproduce untuned ones exactly."""
import numpy as np
import pytest

from oracle.covariance import Cov as OCov
from oracle.pipeline import draw_observations
from paper_2109_11044_amd import cesim, workloads

pytestmark = pytest.mark.gpu


def run(prec, m, torus, params=(), nreal=6, tune=False, cov=(1.5, 1.0, 0.1)):
    import torch
    xy = workloads.uniform_locations(120, seed=21)
    z = draw_observations(xy, OCov(*cov), 0.05, seed=0)
    with cesim.Context(cesim.make_cov(*cov), cesim.unit_square_grid(m, torus), prec) as ctx:
        ctx.offgrid(xy, 16)
        if tune:
            scratch = torch.empty((nreal, m, m), dtype=ctx.dtype, device="cuda")
            ctx.autotune(nreal, scratch)
        for p, v in params:
            ctx.set_param(p, v)
        f = ctx.simulate(nreal, seed=3, first_real=1)
        y = f.clone()
        ctx.condition(z, 0.05, f)
        return y.cpu(), f.cpu()


@pytest.mark.parametrize("prec,m,torus", [("fp64", 128, 256), ("mixed", 128, 256),
                                          ("mixed", 128, 384), ("mixed", 256, 768)])
def test_every_draw_tile_shape_gives_identical_fields(prec, m, torus):
    import torch
    cesim.tune_clear()
    y0, v0 = run(prec, m, torus)
    for rows in (1, 2, 4, 8):
        for cols in (1, 2, 4, 16):
            y, v = run(prec, m, torus, [(cesim.PARAM_DRAW_COLS, cols),
                                       (cesim.PARAM_DRAW_ROWS, rows)])
            assert torch.equal(y, y0) and torch.equal(v, v0), (rows, cols)


@pytest.mark.parametrize("nreal", [6, 300, 600])
def test_gemm_tiles_give_identical_fields(nreal):
    import torch
    cesim.tune_clear()
    _, v1 = run("mixed", 128, 256, [(cesim.PARAM_GEMM_TILE, 1)], nreal=nreal)
    for tile in (2, 3, 4, 5):
        _, v = run("mixed", 128, 256, [(cesim.PARAM_GEMM_TILE, tile)], nreal=nreal)
        assert torch.equal(v1, v), tile


@pytest.mark.parametrize("prec,torus", [("mixed", 384), ("fp64", 256), ("mixed", 256)])
def test_autotune_fills_table_and_keeps_results(prec, torus, tmp_path):
    import torch
    cesim.tune_clear()
    y0, v0 = run(prec, 128, torus)
    y1, v1 = run(prec, 128, torus, tune=True)
    assert cesim.tune_entries() == (2 if prec == "mixed" else 1)
    assert torch.equal(y0, y1) and torch.equal(v0, v1)
    path = tmp_path / "tune.jsonl"
    cesim.tune_save(str(path))
    cesim.tune_clear()
    cesim.tune_load(str(path))
    y2, v2 = run(prec, 128, torus)                  # table entries in force
    assert torch.equal(y0, y2) and torch.equal(v0, v2)
    cesim.tune_clear()


def test_batch_autotune_reproduces_untuned_batch():
    import torch
    from test_gpu_batch import make_events
    cesim.tune_clear()
    evs, _ = make_events()
    with cesim.Batch(evs, "mixed") as b:
        ref = [f.cpu() for f in b.run(3)]
    with cesim.Batch(evs, "mixed", autotune=True) as b:
        got = [f.cpu() for f in b.run(3)]
    assert cesim.tune_entries() > 0
    for a, r in zip(got, ref):
        assert torch.equal(a, r)
    cesim.tune_clear()
