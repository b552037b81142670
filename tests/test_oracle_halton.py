"""Pins of the oracle's radical inversion in prime bases and the Halton sequence (Sec. 2.2)."""

from fractions import Fraction

import numpy as np
import pytest

from oracle import digital, halton


def test_primes_and_max_powers():
    assert halton.primes(12) == [2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37]
    assert halton.primes(64)[-1] == 311
    assert halton.max_power(2) == 2 ** 31
    assert halton.max_power(3) == 3486784401  # the listing's reduction constant for phi_3
    assert halton.max_power(5) == 5 ** 13
    for b in halton.primes(64):
        q = halton.max_power(b)
        assert q <= 0xFFFFFFFF < q * b


def test_faure_permutations():
    assert halton.faure_permutation(2) == [0, 1]
    assert halton.faure_permutation(3) == [0, 1, 2]
    assert halton.faure_permutation(4) == [0, 2, 1, 3]
    assert halton.faure_permutation(5) == [0, 3, 2, 1, 4]  # the paper's example
    for b in range(2, 320):
        s = halton.faure_permutation(b)
        assert sorted(s) == list(range(b)) and s[0] == 0
        if b % 2 == 1 and b > 2:
            assert s[(b - 1) // 2] == (b - 1) // 2  # the inserted middle value


def test_two_digit_table_of_the_listing_base3():
    """The listing's base-9 table inverts two base-3 digits at once: entry t = a0 + 3 a1 holds
    3 a0 + a1, so phi_3(t) = table[t] / 9 for t < 9."""
    table = [0, 3, 6, 1, 4, 7, 2, 5, 8]
    for t in range(9):
        assert halton.radical_inverse_u32(t, 3) == (table[t] << 32) // 9


def test_two_digit_faure_table_base5():
    """sigma_5 x sigma_5 as printed: entry (a0, a1) = 5 sigma(a0) + sigma(a1).  The printed
    second row (25, 28, 27, 26, 29) exceeds 24; with sigma(1) = 3 it reads 15, 18, 17, 16, 19."""
    sig = halton.faure_permutation(5)
    rows = [[0, 3, 2, 1, 4], [15, 18, 17, 16, 19], [10, 13, 12, 11, 14], [5, 8, 7, 6, 9], [20, 23, 22, 21, 24]]
    for a0 in range(5):
        for a1 in range(5):
            assert rows[a0][a1] == 5 * sig[a0] + sig[a1]
            assert halton.radical_inverse_u32(a0 + 5 * a1, 5, sig) == (rows[a0][a1] << 32) // 25


def test_halton_first_points():
    # textbook values: (0,0), (1/2,1/3), (1/4,2/3), (3/4,1/9), (1/8,4/9), (5/8,7/9)
    pts = halton.halton_points(2, 0, 6)
    want = [(Fraction(0), Fraction(0)), (Fraction(1, 2), Fraction(1, 3)), (Fraction(1, 4), Fraction(2, 3)),
            (Fraction(3, 4), Fraction(1, 9)), (Fraction(1, 8), Fraction(4, 9)), (Fraction(5, 8), Fraction(7, 9))]
    for k, (x, y) in enumerate(want):
        assert int(pts[0, k]) == (x.numerator << 32) // x.denominator
        assert int(pts[1, k]) == (y.numerator << 32) // y.denominator


def test_base2_is_van_der_corput_of_the_reduced_index():
    rng = np.random.default_rng(4)
    for i in rng.integers(0, 2 ** 32, 100):
        assert halton.radical_inverse_u32(int(i), 2) == int(digital.radical_inverse_base2(np.uint64(int(i) % 2 ** 31)))


@pytest.mark.parametrize("b", [3, 5, 7, 11])
@pytest.mark.parametrize("mode", ["identity", "faure", "linear"])
def test_first_b_power_points_stratify(b, mode):
    """phi_{b,sigma} of i < b^m is a permutation of {k / b^m}: one point per cell."""
    m = 3 if b < 11 else 2
    sig = halton.digit_permutation(b, mode, factor=2)
    got = sorted(halton.radical_inverse_u32(i, b, sig) for i in range(b ** m))
    assert got == [(k << 32) // b ** m for k in range(b ** m)]


def test_index_reduction_wraps():
    for b in (3, 7, 101):
        q = halton.max_power(b)
        for i in (0, 1, 5, 12345):
            if i + q <= 0xFFFFFFFF:
                assert halton.radical_inverse_u32(i + q, b) == halton.radical_inverse_u32(i, b)


def test_linear_scramble_is_digitwise():
    b, f = 7, 3
    sig = halton.digit_permutation(b, "linear", f)
    assert sig == [(f * a) % b for a in range(b)]
    # digits 2, 5, 1 (i = 2 + 5*7 + 1*49) map to sigma(2)/7 + sigma(5)/49 + sigma(1)/343
    i = 2 + 5 * 7 + 49
    want = Fraction(sig[2], 7) + Fraction(sig[5], 49) + Fraction(sig[1], 343)
    assert halton.radical_inverse_u32(i, b, sig) == (want.numerator << 32) // want.denominator
