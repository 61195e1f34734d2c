"""Pins of the oracle's circulant-embedding setup and draw (Section 1;
Section 2.1 item (a)): brute-force DFT, trace, evenness and the exactness of
the draw's covariance."""
import numpy as np
import pytest

from oracle import ce, philox
from oracle.covariance import Cov, cross_covariance
from oracle.pipeline import Grid, draw_matrix, setup


def brute_dft2(c):
    t2, t1 = c.shape
    q2, q1 = np.meshgrid(np.arange(t2), np.arange(t1), indexing="ij")
    lam = np.empty((t2, t1), dtype=complex)
    for k2 in range(t2):
        for k1 in range(t1):
            ph = np.exp(-2j * np.pi * (k1 * q1 / t1 + k2 * q2 / t2))
            lam[k2, k1] = (c * ph).sum()
    return lam


def test_smooth_sizes_and_ladder():
    assert ce.next_smooth(127) == 128 and ce.next_smooth(129) == 135
    assert ce.next_smooth(7 * 11) == 80
    assert ce.torus_ladder(64, 64) == [(128, 128), (192, 192), (256, 256),
                                       (384, 384), (512, 512)]
    assert ce.torus_ladder(2048, 2048) == [(4096, 4096), (6144, 6144), (8192, 8192)]
    assert ce.torus_ladder(100, 70)[0] == (200, 144)   # 140 = 4*5*7 is not smooth


@pytest.mark.parametrize("cov,t1,t2", [
    (Cov(0.5, 1.0, 0.3), 8, 8),
    (Cov(1.5, 2.0, 0.4, 2.0, 0.7), 6, 10),
    (Cov(1.0, 1.0, 0.25, 1.5, 2.0), 9, 12),
])
def test_eigenvalues_vs_brute_force_dft(cov, t1, t2):
    c = ce.torus_base(cov, 0.1, 0.13, t1, t2)
    lam, info = ce.eigenvalues(c)
    bf = brute_dft2(c)
    scale = np.abs(bf).max()
    assert np.max(np.abs(lam - bf.real)) < 1e-13 * scale
    assert np.max(np.abs(bf.imag)) < 1e-13 * scale       # spectrum is real
    assert info["lam_sum"] == pytest.approx(t1 * t2 * cov.sigma2, rel=1e-13)
    # evenness lambda(k) = lambda(-k)
    neg = lam[(-np.arange(t2)) % t2][:, (-np.arange(t1)) % t1]
    assert np.max(np.abs(lam - neg)) < 1e-13 * scale


def test_torus_base_values():
    cov = Cov(0.5, 1.0, 0.2)
    c = ce.torus_base(cov, 0.1, 0.1, 8, 8)
    assert c[0, 0] == 1.0
    assert c[0, 3] == pytest.approx(np.exp(-0.3 / 0.2), rel=1e-15)
    assert c[0, 5] == pytest.approx(np.exp(-0.3 / 0.2), rel=1e-15)   # wrapped
    assert c[0, 4] == pytest.approx(np.exp(-0.4 / 0.2), rel=1e-15)   # Nyquist
    assert c[2, 7] == pytest.approx(np.exp(-np.hypot(0.1, 0.2) / 0.2), rel=1e-15)


@pytest.mark.parametrize("cov,m,t", [
    (Cov(0.5, 1.0, 0.3), 4, None),
    (Cov(0.5, 1.0, 0.5), 6, None),
    (Cov(1.5, 1.0, 0.2), 6, 18),                 # padded, radix-3 torus
    (Cov(1.0, 1.7, 0.25), 8, None),
    (Cov(0.5, 1.0, 0.4, 2.0, 0.5), 6, 15),        # anisotropic, odd torus
    (Cov(1.5, 1.0, 0.3, 3.0, 1.2), 5, None),      # anisotropic, Nyquist lines
])
def test_draw_is_exact(cov, m, t):
    """B B^T equals the grid covariance when no eigenvalue is clamped."""
    g = Grid.unit_square(m)
    t1, t2, s, info = setup(cov, g, t, t)
    assert info["lam_min"] >= 0.0
    Bre = draw_matrix(s, m, m, 0)        # realization 2P from (eps_2P, eps_2P+1)
    Bim = draw_matrix(s, m, m, 1)        # realization 2P + 1
    P = g.points()
    K = cross_covariance(P, P, cov)
    assert np.max(np.abs(Bre @ Bre.T - K)) < 1e-12 * cov.sigma2
    assert np.max(np.abs(Bim @ Bim.T - K)) < 1e-12 * cov.sigma2
    # the two members of a pair are uncorrelated (jointly Gaussian: independent)
    assert np.max(np.abs(Bre @ Bim.T)) < 1e-12 * cov.sigma2


def test_negative_eigenvalues_detected_and_ladder_moves_on():
    # Matern 1.5 with a long range on a small torus has negative eigenvalues.
    cov = Cov(1.5, 1.0, 0.3)
    g = Grid.unit_square(32)
    with pytest.raises(ce.NegativeEigenvalue):
        setup(cov, g, 64, 64)
    t1, t2, s, info = setup(cov, g)
    assert t1 > 64 and info["lam_min"] >= -1e-12 * info["lam_max"]


def test_acceptance_checks_reality_and_trace():
    """A valid spectrum passes all three checks; a base that is not even (an
    FFT or base bug) has a non-real spectrum and is refused; so is a spectrum
    whose sum misses the trace identity sum(lambda) = N C(0)."""
    cov = Cov(0.5, 1.0, 0.1)
    g = Grid.unit_square(16)
    c = ce.torus_base(cov, g.dx, g.dy, 32, 32)
    lam, info = ce.eigenvalues(c)
    assert ce.accept(info)
    assert info["trace"] == 32 * 32 * 1.0
    assert abs(info["lam_sum"] - info["trace"]) < 1e-12 * info["trace"]
    assert info["max_imag"] < 1e-13 * info["lam_max"]
    odd = c.copy()
    odd[0, 1] += 1e-3                     # breaks c[q] = c[-q]
    _, oinfo = ce.eigenvalues(odd)
    assert oinfo["lam_min"] >= -1e-12 * oinfo["lam_max"]
    assert oinfo["max_imag"] > 1e-12 * oinfo["lam_max"] and not ce.accept(oinfo)
    bad = dict(info, lam_sum=info["trace"] * (1 + 2e-9))
    assert not ce.accept(bad)
    assert ce.accept(dict(info, lam_sum=info["trace"] * (1 + 5e-10)))


def test_matern1_range015_needs_padding():
    """nu = 1, theta = 0.15 on a 256^2 unit-square grid: the 512 torus has a
    negative spectrum, 768 is the first accepted size."""
    cov = Cov(1.0, 1.0, 0.15)
    g = Grid.unit_square(256)
    lam, info = ce.eigenvalues(ce.torus_base(cov, g.dx, g.dy, 512, 512))
    assert info["lam_min"] < -1e-12 * info["lam_max"]
    t1, t2, _, _ = setup(cov, g)
    assert (t1, t2) == (768, 768)


def test_unconditional_moments_monte_carlo():
    """Empirical covariances of Philox-driven draws match C(h) (|z| < 4)."""
    cov = Cov(0.5, 1.0, 0.3)
    m = 8
    g = Grid.unit_square(m)
    t1, t2, s, _ = setup(cov, g)
    R = 4000
    y = ce.ce_draw(s, 21, range(R), m, m).reshape(R, -1)
    P = g.points()
    K = cross_covariance(P, P, cov)
    for (i, j) in [(0, 0), (0, 1), (9, 27), (5, 60), (63, 63), (0, 63)]:
        prod = y[:, i] * y[:, j]
        zsc = (prod.mean() - K[i, j]) / (prod.std() / np.sqrt(R))
        assert abs(zsc) < 4, (i, j, zsc)
    assert abs(y.mean()) < 4 / np.sqrt(R)
    # the members of a pair (2P, 2P + 1) are uncorrelated at every lag
    ye, yo = y[0::2], y[1::2]
    for (i, j) in [(0, 0), (9, 27), (63, 0), (20, 21)]:
        prod = ye[:, i] * yo[:, j]
        zsc = prod.mean() / (prod.std() / np.sqrt(ye.shape[0]))
        assert abs(zsc) < 4, (i, j, zsc)


def test_realization_depends_only_on_its_index():
    """Pairs are absolute (P = r // 2), so any batching gives the same fields,
    including calls that start or end inside a pair."""
    cov = Cov(1.5, 1.0, 0.2)
    g = Grid.unit_square(6)
    t1, t2, s, _ = setup(cov, g)
    full = ce.ce_draw(s, 5, range(7), 6, 6, event=2)
    for lo, hi in [(1, 4), (3, 4), (4, 7), (0, 1), (5, 6)]:
        assert np.array_equal(ce.ce_draw(s, 5, range(lo, hi), 6, 6, event=2), full[lo:hi])
    assert not np.allclose(ce.ce_draw(s, 5, range(2), 6, 6, event=3), full[:2])
