"""Pins of the oracle's covariance model (Section 3.3) against closed forms,
an independent Bessel evaluation and values printed in the paper."""
import os

import mpmath
import numpy as np
import pytest
from scipy.integrate import quad
from scipy.special import gamma as G
from scipy.special import kv

from oracle.covariance import Cov, covariance, matern_correlation

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def bessel_form(x, nu):
    t = np.sqrt(2 * nu) * x
    return 2 ** (1 - nu) / G(nu) * t ** nu * kv(nu, t)


@pytest.mark.parametrize("nu", [0.5, 1.5])
def test_closed_forms_match_bessel_definition(nu):
    x = np.concatenate([np.logspace(-6, 1.5, 400), [0.1, 1.0, 2.0]])
    got = matern_correlation(x, nu)
    want = bessel_form(x, nu)
    assert np.max(np.abs(got - want) / np.abs(want)) < 1e-12


def test_nu1_matches_mpmath_and_integral():
    x = np.concatenate([np.logspace(-8, np.log10(400.0), 300)])
    got = matern_correlation(x, 1.0)
    mp = np.array([float(mpmath.sqrt(2) * xx * mpmath.besselk(1, mpmath.sqrt(2) * xx))
                   for xx in x])
    assert np.max(np.abs(got - mp) / mp) < 1e-13
    # K_1(t) = int_0^inf exp(-t cosh u) cosh u du, independent of scipy.kv
    for xx in (0.05, 0.7, 3.0):
        t = np.sqrt(2) * xx
        umax = np.arccosh(740.0 / t)      # integrand below 1e-300 beyond
        k1, _ = quad(lambda u: np.exp(-t * np.cosh(u)) * np.cosh(u), 0, umax,
                     epsabs=0, epsrel=1e-13, limit=200)
        assert abs(matern_correlation(np.array([xx]), 1.0)[0] - t * k1) < 1e-11


def test_value_at_zero_is_sill():
    for nu in (0.5, 1.0, 1.5):
        cov = Cov(nu, 2.5, 0.3)
        assert covariance(0.0, 0.0, cov) == pytest.approx(2.5, rel=0, abs=0)


def test_printed_exponential_ranges():
    """theta with rho(d / theta) = 0.05 rounds to the printed values."""
    rows = np.loadtxt(os.path.join(GOLD, "exponential_ranges.txt"))
    for d, theta_printed in rows:
        lo, hi = 1.0, 100.0
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            r = covariance(d, 0.0, Cov(0.5, 1.0, mid))
            lo, hi = (mid, hi) if r < 0.05 else (lo, mid)
        assert round(0.5 * (lo + hi), 2) == pytest.approx(theta_printed)


def test_anisotropy_axes_and_evenness():
    cov = Cov(1.5, 1.3, 0.2, aniso_ratio=2.5, aniso_angle=0.6)
    d = np.linspace(0.0, 0.5, 11)
    c, s = np.cos(0.6), np.sin(0.6)
    along = covariance(d * c, d * s, cov)
    across = covariance(-d * s, d * c, cov)
    assert np.allclose(along, 1.3 * matern_correlation(d / 0.2, 1.5), rtol=1e-14)
    assert np.allclose(across, 1.3 * matern_correlation(2.5 * d / 0.2, 1.5), rtol=1e-14)
    rng = np.random.default_rng(0)
    h = rng.normal(size=(2, 50)) * 0.2
    assert np.allclose(covariance(h[0], h[1], cov), covariance(-h[0], -h[1], cov),
                       rtol=1e-15)
    # not symmetric under reflecting one axis when anisotropic
    assert not np.allclose(covariance(h[0], h[1], cov), covariance(-h[0], h[1], cov))
    iso = Cov(0.5, 1.0, 0.2)
    assert np.allclose(covariance(h[0], h[1], iso),
                       np.exp(-np.hypot(h[0], h[1]) / 0.2), rtol=1e-14)
