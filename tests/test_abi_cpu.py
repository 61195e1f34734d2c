"""CPU checks of the C ABI: the library loads, exports every declared
symbol, its host-evaluable code (covariance, Philox) agrees with the oracle,
and argument errors are reported before any device work."""
import ctypes
import os
import re

import mpmath
import numpy as np
import pytest

from oracle import philox
from oracle.covariance import Cov, covariance
from paper_2109_11044_amd import cesim

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "cesim.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(\w+)\s*\([^;{]*\)\s*;", src)))


def test_library_exports_every_declared_symbol():
    names = declared_functions()
    assert "ce_setup" in names and "condition" in names and len(names) >= 12
    L = cesim.lib()
    for n in names:
        assert hasattr(L, n), n
    assert set(cesim.EXPORTS) == set(names)


@pytest.mark.parametrize("nu", [0.5, 1.0, 1.5])
@pytest.mark.parametrize("aniso", [(1.0, 0.0), (2.5, 0.7), (1.7, 2.9)])
def test_library_covariance_matches_oracle(nu, aniso):
    c = cesim.make_cov(nu, 1.3, 0.2, *aniso)
    rng = np.random.default_rng(0)
    hx, hy = rng.normal(size=(2, 2000)) * 0.6
    hx[:5] = 0.0
    hy[:5] = [0.0, 1e-9, 0.3, -0.3, 1e-3]
    got = cesim.covariance_host(c, hx, hy)
    ref = covariance(hx, hy, Cov(nu, 1.3, 0.2, *aniso))
    mask = ref > 1e-290
    # a relative rounding error e of the lag length moves rho by about x e,
    # x = d / theta (both sides round the anisotropic metric differently)
    from oracle.covariance import lag_distance
    x = lag_distance(hx, hy, Cov(nu, 1.3, 0.2, *aniso)) / 0.2
    tol = 4e-15 * (1.0 + x[mask])
    assert np.all(np.abs(got[mask] - ref[mask]) / ref[mask] < tol)


def test_library_bessel_k1_against_mpmath():
    """nu = 1 goes through the library's own K_1 (series / quadrature /
    asymptotic branches)."""
    c = cesim.make_cov(1.0, 1.0, 1.0 / np.sqrt(2.0))   # t = sqrt(2) d / theta = 2 d
    t = np.concatenate([np.logspace(-9, np.log10(650), 700), [2.0, 30.0, 30.000001]])
    got = cesim.covariance_host(c, t / 2.0, np.zeros_like(t))
    ref = np.array([float(mpmath.mpf(x) * mpmath.besselk(1, x)) for x in t])
    # t K1(t) has argument condition number about t; the lag t/2 is
    # rescaled by 1/theta = sqrt(2) in floating point before K1 sees it
    assert np.all(np.abs(got - ref) / ref < 5e-15 + 1e-15 * t)


def test_library_philox_matches_oracle():
    ctr = np.arange(0, 4096, 7)
    for seed, c1, c2, c3 in [(0, 0, 0, 0), (2, 17, 0, 1), (2 ** 63 + 12345, 999, 3, 2)]:
        w = cesim.philox_host(seed, ctr, c1, c2, c3)
        assert np.array_equal(w, philox.raw_words(seed, ctr, c1, c2, c3))


def test_setup_argument_errors_without_device():
    L = cesim.lib()
    h = ctypes.c_void_p()
    good_cov = cesim.make_cov(0.5, 1.0, 0.1)
    good_grid = cesim.unit_square_grid(16)
    bad = [
        (cesim.make_cov(0.7, 1.0, 0.1), good_grid, 0),
        (cesim.make_cov(0.5, -1.0, 0.1), good_grid, 0),
        (cesim.make_cov(0.5, 1.0, 0.0), good_grid, 0),
        (cesim.make_cov(0.5, 1.0, 0.1, 0.5), good_grid, 0),
        (good_cov, cesim.Grid(1, 16, 0, 0, 0.1, 0.1, 0, 0), 0),
        (good_cov, cesim.Grid(16, 16, 0, 0, 0.0, 0.1, 0, 0), 0),
        (good_cov, cesim.Grid(16, 16, 0, 0, 0.1, 0.1, 20, 32), 0),   # torus < 2m-1
        (good_cov, cesim.Grid(16, 16, 0, 0, 0.1, 0.1, 49, 49), 0),   # 7^2 not smooth
        (good_cov, good_grid, 7),                                    # precision
    ]
    for cov, grid, prec in bad:
        st = L.ce_setup(ctypes.byref(cov), ctypes.byref(grid), prec, None, ctypes.byref(h))
        assert st == 1 and not h.value
    assert L.ce_setup(None, ctypes.byref(good_grid), 0, None, ctypes.byref(h)) == 1
    assert L.ce_simulate(None, 1, 0, 0, None) == 1
    assert L.condition(None, None, 0.0, None) == 1
    assert L.cesim_status_string(2).decode().startswith("negative")
    L.ce_destroy(None)


def test_tuning_table_save_load_round_trip(tmp_path):
    cesim.tune_clear()
    src = tmp_path / "in.jsonl"
    src.write_text('{"key": "drawAB p1 2048x2048", "v": [2, 8, 0]}\n'
                   '{"key": "gemm s0 nu0 M1048576 n10 R1024", "v": [2, 0, 0]}\n')
    cesim.tune_load(str(src))
    assert cesim.tune_entries() == 2
    out = tmp_path / "out.jsonl"
    cesim.tune_save(str(out))
    assert sorted(out.read_text().splitlines()) == sorted(src.read_text().splitlines())
    bad = tmp_path / "bad.jsonl"
    bad.write_text('{"key": "drawAB p1 64x64", "v": [1, 1, 0]}\nnot json\n')
    with pytest.raises(cesim.CesimError) as e:
        cesim.tune_load(str(bad))
    assert e.value.name == "INVALID_ARG"
    assert cesim.tune_entries() == 3          # the line before the bad one is kept
    with pytest.raises(cesim.CesimError):
        cesim.tune_load(str(tmp_path / "missing.jsonl"))
    cesim.tune_clear()
    assert cesim.tune_entries() == 0
