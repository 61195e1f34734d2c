"""Error paths of the C ABI on the GPU: every failure is a status code and
the context stays usable afterwards."""
import ctypes

import numpy as np
import pytest

from paper_2109_11044_amd import cesim

pytestmark = pytest.mark.gpu


def status_of(fn, *a):
    with pytest.raises(cesim.CesimError) as e:
        fn(*a)
    return e.value.name


def test_forced_torus_with_negative_eigenvalues():
    name = status_of(cesim.Context, cesim.make_cov(1.5, 1.0, 0.3), cesim.unit_square_grid(32, 64))
    assert name == "NEGATIVE_EIGENVALUE"


def test_offgrid_argument_errors():
    with cesim.Context(cesim.make_cov(0.5, 1.0, 0.1), cesim.unit_square_grid(8)) as ctx:
        ok = np.array([[0.5, 0.5], [1.0, 1.0], [0.0, 0.0]])
        assert status_of(ctx.offgrid, ok, 25) == "INVALID_ARG"
        assert status_of(ctx.offgrid, ok, 100) == "INVALID_ARG"
        assert status_of(ctx.offgrid, np.array([[0.5, 1.0 + 1e-6]]), 16) == "OBS_OUTSIDE_GRID"
        assert status_of(ctx.offgrid, np.array([[np.nan, 0.5]]), 16) == "OBS_OUTSIDE_GRID"
        assert status_of(ctx.offgrid, np.array([[-1e-6, 0.5]]), 16) == "OBS_OUTSIDE_GRID"
    with cesim.Context(cesim.make_cov(0.5, 1.0, 0.1), cesim.unit_square_grid(6)) as ctx:
        assert status_of(ctx.offgrid, np.array([[0.5, 0.5]]), 64) == "INVALID_ARG"
        ctx.offgrid(np.array([[0.5, 0.5]]), 36)            # 6 x 6 window fits exactly


def test_out_of_order_calls_and_recovery():
    import torch
    with cesim.Context(cesim.make_cov(0.5, 1.0, 0.2), cesim.unit_square_grid(16)) as ctx:
        f = torch.zeros((2, 16, 16), dtype=torch.float64, device="cuda")
        ctx.nobs = 2
        assert status_of(ctx.condition, np.zeros(2), 0.1, f) == "BAD_STATE"   # no offgrid
        xy = np.array([[0.3, 0.3], [0.3, 0.3]])                                 # duplicates
        ctx.offgrid(xy, 16)
        assert status_of(ctx.condition, np.zeros(2), 0.1, f) == "BAD_STATE"   # no simulate
        ctx.simulate(2, 1, out=f)
        assert status_of(ctx.condition, np.zeros(2), 0.0, f) == "NOT_POSITIVE_DEFINITE"
        assert status_of(ctx.condition, np.zeros(2), -1.0, f) == "INVALID_ARG"
        assert status_of(ctx.condition, np.array([0.0, np.nan]), 0.1, f) == "INVALID_ARG"
        ctx.condition(np.array([0.5, 0.5]), 0.1, f)                            # recovers
        assert torch.isfinite(f).all()
        # a conditioned batch is not conditioned twice; a new draw re-arms it
        assert status_of(ctx.condition, np.array([0.5, 0.5]), 0.1, f) == "BAD_STATE"
        ctx.simulate(2, 1, out=f)
        ctx.condition(np.array([0.5, 0.5]), 0.1, f)
    L = cesim.lib()
    assert L.ce_simulate(None, 1, 0, 0, None) == 1


def test_simulate_argument_errors():
    import torch
    with cesim.Context(cesim.make_cov(0.5, 1.0, 0.2), cesim.unit_square_grid(16)) as ctx:
        f = torch.zeros((2, 16, 16), dtype=torch.float64, device="cuda")
        L = cesim.lib()
        assert L.ce_simulate(ctx._h, 0, 1, 0, ctypes.c_void_p(f.data_ptr())) == 1
        assert L.ce_simulate(ctx._h, 1, 1, -1, ctypes.c_void_p(f.data_ptr())) == 1
        assert L.ce_simulate(ctx._h, 1, 1, 0, None) == 1
        assert L.ce_set_param(ctx._h, 99, 1) == 1
        assert L.ce_set_param(ctx._h, cesim.PARAM_GEMM_TILE, 6) == 1
