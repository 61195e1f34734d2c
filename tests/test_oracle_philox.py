"""Checks of the oracle's Philox4x32-10 stream.

The generator is pinned to the known-answer vectors published with its
reference implementation (tests/golden/philox4x32_10_kat.txt), which both the
oracle and the library's own C++ implementation must reproduce bit for bit;
further checks are a second, scalar, pure-integer implementation, the
statistics of the output and its behaviour as a keyed bijection.  Bit-exact
agreement of the GPU's words with the oracle is checked by the GPU tests."""
import os

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


GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def kat_vectors():
    out = []
    with open(GOLDEN) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                v = [int(x, 16) for x in line.split()]
                out.append((v[:4], v[4:6], v[6:]))
    return out


def test_known_answer_vectors_oracle():
    vecs = kat_vectors()
    assert len(vecs) == 3
    for ctr, key, want in vecs:
        got = philox.philox4x32_10(*(np.uint64(c) for c in ctr), *key)
        assert [int(x) for x in got] == want
        assert scalar_philox(ctr, key) == want


def test_known_answer_vectors_library():
    """The library's host copy of its Philox source, keyed by the 64-bit seed
    k0 | k1 << 32 (no GPU needed)."""
    from paper_2109_11044_amd import cesim
    for ctr, key, want in kat_vectors():
        seed = key[0] | (key[1] << 32)
        w = cesim.philox_host(seed, np.array([ctr[0]], dtype=np.uint32), ctr[1], ctr[2], ctr[3])
        assert [int(x) for x in w[0]] == want


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
