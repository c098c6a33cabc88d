"""Coefficient quantisation of the mixed-precision inner solve (oracle side).

The mixed-precision policy keeps the outer operator in float64 and runs the
inner shifted solves on a copy of kappa rounded to float32 or to bfloat16.
These functions produce that rounded copy from the float64 field, written from
the IEEE-754 definitions: float32 by numpy's round-to-nearest-even cast, and
bfloat16 as the upper 16 bits of the float32 pattern after round-to-nearest-
even on the discarded 16 bits.  The oracle then runs its float64 arithmetic on
the rounded field, so that a GPU/oracle comparison isolates the arithmetic
precision from the coefficient storage.

Pins (tests/test_oracle_precision.py): exact values of representable numbers,
ties to even, and the 2^-8 relative rounding bound (8-bit significand).
"""

from __future__ import annotations

import numpy as np


def to_float32(x) -> np.ndarray:
    return np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float64)


def to_bfloat16(x) -> np.ndarray:
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lower = u & 0xFFFF
    upper = u >> 16
    # round to nearest, ties to even on the kept 16 bits
    round_up = (lower > 0x8000) | ((lower == 0x8000) & ((upper & 1) == 1))
    upper = upper + round_up.astype(np.uint64)
    out = (upper << 16).astype(np.uint32).view(np.float32)
    return out.astype(np.float64)
