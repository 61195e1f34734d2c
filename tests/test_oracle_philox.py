"""Checks of the oracle's Philox4x32-10 stream.

No published known-answer vectors are available offline, so the generator is
checked by a second, scalar, pure-integer implementation, by the statistics
of its output and by its behaviour as a keyed bijection.  Bit-exact agreement
with the HIP implementation (written separately in C++) is checked by the GPU
tests."""
import numpy as np
import pytest
from scipy import stats

from oracle import philox


def scalar_philox(ctr, key):
    c = list(ctr)
    k0, k1 = key
    for rnd in range(10):
        if rnd:
            k0 = (k0 + 0x9E3779B9) % 2 ** 32
            k1 = (k1 + 0xBB67AE85) % 2 ** 32
        p0 = 0xD2511F53 * c[0]
        p1 = 0xCD9E8D57 * c[2]
        c = [(p1 >> 32) ^ c[1] ^ k0, p1 % 2 ** 32, (p0 >> 32) ^ c[3] ^ k1,
             p0 % 2 ** 32]
    return c


def test_vectorised_matches_scalar():
    rng = np.random.default_rng(5)
    ctr = rng.integers(0, 2 ** 32, size=(64, 4), dtype=np.uint64)
    key = (0xDEADBEEF, 0x01234567)
    out = np.stack(philox.philox4x32_10(ctr[:, 0], ctr[:, 1], ctr[:, 2], ctr[:, 3],
                                        *key), axis=1)
    for i in range(64):
        assert list(out[i]) == scalar_philox([int(x) for x in ctr[i]], key)
    # the all-ones edge
    o = philox.philox4x32_10(*(np.uint64(2 ** 32 - 1),) * 4, 2 ** 32 - 1, 2 ** 32 - 1)
    assert [int(x) for x in o] == scalar_philox([2 ** 32 - 1] * 4, (2 ** 32 - 1,) * 2)


def test_uniformity_and_normal_moments():
    w = philox.raw_words(7, np.arange(50000), 3, 0, 0).reshape(-1)
    hist = np.bincount((w >> np.uint32(24)).astype(np.int64), minlength=256)
    assert stats.chisquare(hist).pvalue > 1e-4
    z = philox.normals(11, 400000, 0)
    assert abs(z.mean()) < 5 / np.sqrt(z.size)
    assert abs(z.var() - 1) < 5 * np.sqrt(2 / z.size)
    assert stats.kstest(z[:100000], "norm").pvalue > 1e-4
    u = philox.uniforms(w)
    assert u.min() > 0 and u.max() < 1


def test_streams_are_distinct_and_uncorrelated():
    a = philox.normals(3, 20000, 0, 0, 0)
    b = philox.normals(3, 20000, 1, 0, 0)
    c = philox.normals(3, 20000, 0, 0, 1)
    d = philox.normals(4, 20000, 0, 0, 0)
    for x in (b, c, d):
        assert abs(np.corrcoef(a, x)[0, 1]) < 5 / np.sqrt(a.size)
    # avalanche: one counter bit flips about half of the output bits
    base = philox.raw_words(9, np.arange(2000), 0, 0, 0)
    flip = philox.raw_words(9, np.arange(2000) ^ 1, 0, 0, 0)
    bits = np.unpackbits((base ^ flip).view(np.uint8)).mean()
    assert 0.47 < bits < 0.53


def test_bijection_on_a_sample():
    w = philox.raw_words(1, np.arange(1 << 16), 0, 0, 0)
    as_int = (w[:, 0].astype(np.uint64) << np.uint64(32)) | w[:, 1].astype(np.uint64)
    assert np.unique(as_int).size == 1 << 16


def test_element_to_block_mapping():
    z = philox.normals(2, 10, 5, 0, 0)
    u = philox.uniforms(philox.raw_words(2, [2], 5, 0, 0))[0]
    r = np.sqrt(-2 * np.log(u[2]))
    assert z[8] == pytest.approx(np.sqrt(-2 * np.log(u[0])) * np.cos(2 * np.pi * u[1]), rel=1e-15)
    assert z[9] == pytest.approx(np.sqrt(-2 * np.log(u[0])) * np.sin(2 * np.pi * u[1]), rel=1e-15)
    zz = philox.normals(2, 12, 5, 0, 0)
    assert zz[10] == pytest.approx(r * np.cos(2 * np.pi * u[3]), rel=1e-15)


def test_event_word_selects_an_independent_stream():
    from oracle import philox
    a0 = philox.torus_noise(5, 8, 8, [0, 1])
    assert np.array_equal(a0, philox.torus_noise(5, 8, 8, [0, 1], 0))
    a1 = philox.torus_noise(5, 8, 8, [0, 1], 1)
    assert not np.any(a0 == a1)
    w0 = philox.raw_words(5, np.arange(4), 0, 0, philox.STREAM_OFFGRID)
    w1 = philox.raw_words(5, np.arange(4), 0, 1, philox.STREAM_OFFGRID)
    assert not np.any(w0 == w1)
