"""Pins of the oracle's coefficient rounding (IEEE-754 round to nearest even)."""

import numpy as np

from oracle.precision import to_bfloat16, to_float32


def test_bfloat16_exact_and_ties():
    # representable values stay put
    for v in [1.0, 2.0, 0.5, 1.0 + 2 ** -7, 3.0, 50.0, 1024.0]:
        assert to_bfloat16(v) == v
    # halfway between 1 and 1 + 2^-7 rounds to the even mantissa (1.0)
    assert to_bfloat16(1.0 + 2 ** -8) == 1.0
    # halfway between 1 + 2^-7 and 1 + 2^-6 rounds to 1 + 2^-6 (even)
    assert to_bfloat16(1.0 + 3 * 2 ** -8) == 1.0 + 2 ** -6
    # just above half rounds up
    assert to_bfloat16(1.0 + 2 ** -8 + 2 ** -12) == 1.0 + 2 ** -7


def test_bfloat16_relative_bound():
    x = np.random.default_rng(0).lognormal(3.0, 1.5, 100000)
    r = np.abs(to_bfloat16(x) - x) / x
    assert r.max() <= 2.0 ** -8 * (1 + 1e-6)  # unit roundoff of an 8-bit significand
    assert to_float32(np.float64(1) / 3) == np.float32(1) / np.float32(3)
