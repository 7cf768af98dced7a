"""Pins for the oracle's dot product: closed forms, math.fsum on exactly
representable products (correctly rounded reference), exact rationals on
tiny inputs.  CPU only."""
import math
from fractions import Fraction

import numpy as np

import gen
import oracle


def test_closed_forms():
    for n in (0, 1, 7, 1000, 150_000, 1 << 20):
        ones = np.ones(n)
        assert oracle.dot(ones, ones) == float(n)
    n = 1 << 20
    i = np.arange(n, dtype=np.float64)
    assert oracle.dot(i, np.ones(n)) == n * (n - 1) / 2
    alt = np.where(np.arange(n) % 2 == 0, 1.0, -1.0)
    assert oracle.dot(alt, np.ones(n)) == 0.0
    assert oracle.dot(alt, alt) == float(n)


def test_fsum_correctly_rounded_reference():
    """a_i, b_i with 26-bit significands: every product is exact in binary64,
    so math.fsum of the products is the correctly rounded dot; the oracle must
    be within 2 ulp-scale of sum |a_i b_i| (compensated summation)."""
    rng = np.random.default_rng(5)
    n = 150_000
    a = np.round(rng.uniform(-1, 1, n) * 2**25) / 2**25
    b = np.round(rng.uniform(-1, 1, n) * 2**25) / 2**25
    prods = a * b
    assert np.array_equal(prods, np.array([float(Fraction(x) * Fraction(y))
                                           for x, y in zip(a[:100], b[:100])] +
                                          list(prods[100:])))
    ref = math.fsum(prods)
    mag = float(np.sum(np.abs(prods)))
    assert abs(oracle.dot(a, b) - ref) <= 4 * 2.0**-53 * mag
    assert oracle.dot_abs(a, b) == np.sum(np.abs(prods)) or \
        abs(oracle.dot_abs(a, b) - math.fsum(np.abs(prods))) <= 1e-12 * mag


def test_fraction_exact_tiny():
    for seed in range(10):
        a = gen.vector(50, seed)
        b = gen.vector(50, seed + 50)
        exact = sum((Fraction(float(x)) * Fraction(float(y)) for x, y in zip(a, b)),
                    Fraction(0))
        mag = float(np.sum(np.abs(a * b)))
        assert abs(Fraction(oracle.dot(a, b)) - exact) <= Fraction(3 * 2.0**-53 * mag)


def test_symmetry_and_scaling():
    a = gen.vector(10_000, 1)
    b = gen.vector(10_000, 2)
    assert oracle.dot(a, b) == oracle.dot(b, a)
    # scaling by a power of two is exact
    assert oracle.dot(4.0 * a, b) == 4.0 * oracle.dot(a, b)


def test_ill_conditioned_sums_match_fsum():
    """Sums where plain recursive summation loses everything: the oracle must
    agree with math.fsum (the correctly rounded sum of exact products)."""
    cases = [
        [1.0, 1e100, 1.0, -1e100],
        [2.0**53, 1.0, 1.0, 1.0, -2.0**53],
        [1e16, 3.0, -1e16, 5.0, 1e-3],
    ]
    rng = np.random.default_rng(3)
    big = np.concatenate([rng.uniform(-1, 1, 5000) * 2.0**60, np.ones(7)])
    big = np.concatenate([big, -big[:5000]])
    cases.append(list(big))
    for a in cases:
        a = np.array(a, dtype=np.float64)
        b = np.ones_like(a)
        assert oracle.dot(a, b) == math.fsum(a), a[:5]
