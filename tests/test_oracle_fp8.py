"""Pins of the oracle's FP8 e4m3 rounding against the format's definition:
the 256 codes decoded from their bit fields, and brute-force nearest-value
search with ties to the even code."""
import numpy as np

from oracle import round_e4m3


def decode_all():
    """Finite non-negative e4m3 values from the bit fields, by code 0..126
    (code 127 = exponent 15, fraction 7 is NaN; 128.. are the negatives)."""
    vals = []
    for code in range(127):
        e, f = code >> 3, code & 7
        vals.append(f / 8 * 2.0 ** -6 if e == 0 else (1 + f / 8) * 2.0 ** (e - 7))
    return np.array(vals)


V = decode_all()


def brute(x):
    """Nearest finite value by exhaustive search; a tie goes to the even code;
    magnitudes beyond the largest value saturate."""
    a = abs(x)
    if a >= V[-1]:
        q = V[-1]
    else:
        dist = np.abs(V - a)
        best = np.flatnonzero(dist == dist.min())
        q = V[best[0]] if len(best) == 1 else V[[c for c in best if c % 2 == 0][0]]
    return np.copysign(q, x)


def test_code_table():
    assert V[1] == 2.0 ** -9 and V[8] == 2.0 ** -6 and V[-1] == 448.0
    assert np.all(np.diff(V) > 0)


def test_fixed_points():
    for s in (1.0, -1.0):
        assert np.array_equal(round_e4m3(s * V), s * V)


def test_midpoints_tie_to_even():
    mids = (V[:-1] + V[1:]) / 2
    want = np.array([brute(m) for m in mids])
    assert np.array_equal(round_e4m3(mids), want)
    assert np.array_equal(round_e4m3(-mids), -want)
    # e.g. 17 lies between 16 (code 0x58, even) and 18 (odd): rounds to 16
    assert round_e4m3(17.0) == 16.0 and round_e4m3(19.0) == 20.0


def test_random_against_brute_force():
    rng = np.random.default_rng(0)
    mag = 2.0 ** rng.uniform(-12, 10, size=4000)
    x = mag * rng.choice([-1.0, 1.0], size=mag.size)
    want = np.array([brute(v) for v in x])
    assert np.array_equal(round_e4m3(x), want)


def test_saturation_and_special_values():
    assert round_e4m3(463.9) == 448.0 and round_e4m3(464.0) == 448.0
    assert round_e4m3(1e30) == 448.0 and round_e4m3(-500.0) == -448.0
    assert round_e4m3(2.0 ** -10) == 0.0 and round_e4m3(1.5 * 2.0 ** -10) == 2.0 ** -9
    r = round_e4m3(np.array([np.inf, -np.inf, np.nan]))
    assert r[0] == np.inf and r[1] == -np.inf and np.isnan(r[2])
