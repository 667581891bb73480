"""Pins of the oracle's block norm: nu = sqrt_RN(RN(exact sum of squares)).

Independent references: Python's exact rationals (Fraction) for the sum,
and correctly rounded int/int division for the rounding; the square root is
checked against the exact bracketing condition."""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle


def exact_sq(v) -> Fraction:
    return sum((Fraction(float(x)) ** 2 for x in np.ravel(v)), Fraction(0))


def rn(q: Fraction) -> float:
    # Fraction -> float is correctly rounded (int / int true division)
    return q.numerator / q.denominator


def is_rn_sqrt(s: float, r: float) -> bool:
    """r is the correctly rounded square root of s (no ties are possible)."""
    if s == 0.0:
        return r == 0.0
    up = math.nextafter(r, math.inf)
    dn = math.nextafter(r, 0.0)
    R, U, D, S = Fraction(r), Fraction(up), Fraction(dn), Fraction(s)
    lo = ((R + D) / 2) ** 2
    hi = ((R + U) / 2) ** 2
    return lo <= S <= hi


def oracle_sq(v):
    v = np.ascontiguousarray(np.ravel(v), dtype=np.float64)
    sq = np.zeros(1); nu = np.zeros(1)
    import ctypes
    oracle.lib().o_block_sq(v.ctypes.data_as(ctypes.c_void_p), v.shape[0],
                            sq.ctypes.data_as(ctypes.c_void_p), nu.ctypes.data_as(ctypes.c_void_p))
    return float(sq[0]), float(nu[0])


ADVERSARIAL = [
    [0.0, 0.0],
    [1.0],
    [1.0, 2.0 ** -27, 2.0 ** -27],        # 1 + 2^-53: exact midpoint, ties to even -> 1.0
    [1.0, 2.0 ** -27, 2.0 ** -27, 2.0 ** -600],  # just above the midpoint -> rounds up
    [1.0, 2.0 ** -26, 2.0 ** -27, 2.0 ** -27],   # midpoint above an odd value -> rounds up
    [5e-324, 5e-324, 1e-310],             # subnormals only
    [1e-160, 3e-170, 2e-200],             # squares far below the normal range
    [1e150, 1e140, -1e145],               # large magnitudes
    [-3.0, 4.0],                          # 25
    [1.0] * 4096,                         # many equal terms
    list(np.linspace(-1, 1, 64) * 1e-8),
]


@pytest.mark.parametrize("v", ADVERSARIAL)
def test_norm_exact_rounding_adversarial(v):
    sq, nu = oracle_sq(v)
    assert sq == rn(exact_sq(v))
    assert is_rn_sqrt(sq, nu)


def test_midpoint_cases_are_really_distinct():
    # guards the two adversarial cases above: they must round differently
    assert oracle_sq([1.0, 2.0 ** -27, 2.0 ** -27])[0] == 1.0
    assert oracle_sq([1.0, 2.0 ** -27, 2.0 ** -27, 2.0 ** -600])[0] == 1.0 + 2.0 ** -52
    assert oracle_sq([1.0, 2.0 ** -26, 2.0 ** -27, 2.0 ** -27])[0] == 1.0 + 2.0 ** -51


@pytest.mark.parametrize("seed", range(6))
def test_norm_exact_rounding_random(seed):
    rng = np.random.default_rng(seed)
    b = [4, 8, 16, 8, 4, 32][seed]
    scale = np.exp(rng.uniform(-60, 5, size=(b, b)))
    v = rng.standard_normal((b, b)) * scale
    v[rng.random((b, b)) < 0.2] = 0.0
    sq, nu = oracle_sq(v)
    assert sq == rn(exact_sq(v))
    assert is_rn_sqrt(sq, nu)


def test_norm_order_and_transpose_invariant():
    rng = np.random.default_rng(7)
    v = rng.standard_normal((16, 16)) * np.exp(rng.uniform(-30, 0, size=(16, 16)))
    a = oracle_sq(v)
    assert oracle_sq(v.T) == a
    assert oracle_sq(rng.permutation(v.ravel())) == a


def test_norm_batch_matches_single_and_nan():
    rng = np.random.default_rng(3)
    vals = rng.standard_normal((5, 8, 8))
    X = oracle.BSM(40, 8, np.arange(5, dtype=np.int32), np.arange(5, dtype=np.int32), vals)
    sq, nu = oracle.norms(X)
    for k in range(5):
        assert (sq[k], nu[k]) == oracle_sq(vals[k])
    assert math.isnan(oracle_sq([1.0, float("nan")])[0])


def test_exact_sum_nonneg():
    rng = np.random.default_rng(11)
    v = np.abs(rng.standard_normal(1000)) * np.exp(rng.uniform(-40, 40, 1000))
    import ctypes
    v = np.ascontiguousarray(v)
    got = oracle.lib().o_exact_sum_nonneg(v.ctypes.data_as(ctypes.c_void_p), v.shape[0])
    assert got == math.fsum(v)
