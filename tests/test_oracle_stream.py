"""Pins for the uniform stream (oracle.stream).

The stream is numpy's Philox4x64-10.  It is pinned here against an
independent big-integer implementation written from the published
definition of Philox (Salmon, Moraes, Dror & Shaw, SC'11: multipliers
0xD2E7470EE14C6C93 / 0xCA5A826395121157, Weyl key increments
0x9E3779B97F4A7C15 / 0xBB67AE8584CAA73B, ten rounds), with block q of the
stream computed at counter q+1.
"""
import numpy as np

from oracle.stream import array_stream, philox_stream

MASK = (1 << 64) - 1


def philox4x64_10(ctr, key):
    c = list(ctr)
    k0, k1 = key
    for _ in range(10):
        p0 = 0xD2E7470EE14C6C93 * c[0]
        p1 = 0xCA5A826395121157 * c[2]
        c = [(p1 >> 64) ^ c[1] ^ k0, p1 & MASK, (p0 >> 64) ^ c[3] ^ k1, p0 & MASK]
        k0 = (k0 + 0x9E3779B97F4A7C15) & MASK
        k1 = (k1 + 0xBB67AE8584CAA73B) & MASK
    return c


def reference_words(seed, start, n):
    out = []
    for p in range(start, start + n):
        q, i = divmod(p, 4)
        ctr = q + 1
        out.append(philox4x64_10([ctr & MASK, ctr >> 64, 0, 0], (seed & MASK, seed >> 64))[i])
    return out


def test_stream_matches_published_philox():
    for seed in (0, 1, 7, 12345, 2**63 + 11):
        for start in (0, 1, 3, 4, 5, 37, 1000):
            ref = reference_words(seed, start, 9)
            got = philox_stream(seed)(start, 9)
            want = np.array([(w >> 11) * 2.0 ** -53 for w in ref])
            assert np.array_equal(got, want), (seed, start)


def test_uniform_conversion_matches_numpy_generator():
    for seed in (0, 3, 99):
        g = np.random.Generator(np.random.Philox(key=seed))
        assert np.array_equal(philox_stream(seed)(0, 50), g.random(50))


def test_uniforms_in_unit_interval():
    U = philox_stream(5)(0, 100_000)
    assert U.min() >= 0.0 and U.max() < 1.0
    assert abs(U.mean() - 0.5) < 0.01


def test_array_stream():
    s = array_stream([0.1, 0.2, 0.3])
    assert np.array_equal(s(1, 2), [0.2, 0.3])
