"""Pins for the oracle's digital sequences (Sec. 2.2 radical inversion, Sec. 2.3 Eq. ts)."""

import math
import os

import numpy as np

from oracle import digital
from synth import sobol_direction_init

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "sobol_2d_first16.txt")


def _euler_phi(n):
    result, m, q = n, n, 2
    while q * q <= m:
        if m % q == 0:
            while m % q == 0:
                m //= q
            result -= result // q
        q += 1
    if m > 1:
        result -= result // m
    return result


def test_primitive_polynomial_counts_match_number_theory():
    # The number of primitive polynomials of degree d over F_2 is phi(2^d - 1) / d.
    polys = digital.primitive_polynomials(1 + 1 + 2 + 2 + 6 + 6 + 18 + 16 + 48 + 60)
    degs = [p.bit_length() - 1 for p in polys]
    for d in range(1, 11):
        assert degs.count(d) == _euler_phi((1 << d) - 1) // d, d
    assert polys[:6] == [0b11, 0b111, 0b1011, 0b1101, 0b10011, 0b11001]


def test_dimension0_is_van_der_corput():
    i = np.arange(4096, dtype=np.uint64)
    x = digital.digital_point(digital.identity_matrix(), i)
    want = np.array([int(format(int(v), "032b")[::-1], 2) for v in i], dtype=np.uint64)
    assert np.array_equal(x, want)


def test_dimension1_is_pascal_mod2():
    # Sobol' matrix of x + 1 (m_1 = 1) equals the Pascal matrix mod 2, C[r,c] = binom(c,r) mod 2.
    m = digital.direction_numbers(0b11, [1])
    cols = digital.generator_matrix_from_m(m)
    for c in range(32):
        for r in range(32):
            bit = (int(cols[c]) >> (31 - r)) & 1
            assert bit == math.comb(c, r) % 2, (r, c)


def test_textbook_first_points_of_the_2d_sequence():
    mats = digital.sobol_matrices(2, sobol_direction_init(2, 0))
    pts = digital.sobol_points(mats, 0, 16).astype(np.uint64)
    for line in open(GOLDEN):
        if line.startswith("#"):
            continue
        i, a, b = map(int, line.split())
        assert int(pts[0, i]) == a << 28 and int(pts[1, i]) == b << 28, i


def test_worked_direction_numbers():
    # Recurrence of Bratley-Fox / Joe-Kuo for x^d + a_1 x^(d-1) + ... + 1, worked by hand.
    assert digital.direction_numbers(0b1011, [1, 3, 5], 8) == [1, 3, 5, 5, 15, 57, 17, 147]
    assert digital.direction_numbers(0b1101, [1, 3, 5], 8) == [1, 3, 5, 3, 29, 23, 53, 159]
    assert digital.direction_numbers(0b111, [1, 3], 8) == [1, 3, 3, 9, 29, 23, 71, 197]


def test_matrices_are_unit_upper_triangular():
    mats = digital.sobol_matrices(32, sobol_direction_init(32, 0))
    for j in range(32):
        for k in range(32):
            col = int(mats[j, k])
            assert (col >> (31 - k)) & 1 == 1          # diagonal
            assert col & ((1 << (31 - k)) - 1) == 0     # nothing below the diagonal


def net_t_value(x, y, m):
    """Smallest t such that the 2^m points (x, y) form a (t, m, 2)-net in base 2."""
    for t in range(m + 1):
        ok = True
        for q in range(m - t + 1):
            r = m - t - q
            cell = (x >> np.uint64(32 - q) if q else np.zeros_like(x)) * np.uint64(1 << r) + \
                   (y >> np.uint64(32 - r) if r else np.zeros_like(y))
            counts = np.bincount(cell.astype(np.int64), minlength=1 << (m - t))
            if not np.all(counts == (1 << t)):
                ok = False
                break
        if ok:
            return t
    return m + 1


def is_02_net_everywhere(x, y, max_m):
    """Every aligned block of 2^m consecutive points, every m <= max_m, is a (0,m,2)-net."""
    for m in range(max_m + 1):
        n = 1 << m
        for b in range(x.size // n):
            if net_t_value(x[b * n:(b + 1) * n], y[b * n:(b + 1) * n], m) != 0:
                return False
    return True


def test_02_sequence_nets_up_to_m16():
    mats = digital.sobol_matrices(2, sobol_direction_init(2, 0))
    pts = digital.sobol_points(mats, 0, 1 << 16).astype(np.uint64)
    x, y = pts[0], pts[1]
    # All blocks for m <= 10; then the leading blocks for 11..16 (same property, fewer blocks).
    assert is_02_net_everywhere(x[: 1 << 12], y[: 1 << 12], 10)
    for m in range(11, 17):
        for b in range(min(2, (1 << 16) >> m)):
            n = 1 << m
            assert net_t_value(x[b * n:(b + 1) * n], y[b * n:(b + 1) * n], m) == 0, (m, b)


def test_pair_t_values_within_sobol_bound():
    # t(pair) <= (deg p_a - 1) + (deg p_b - 1), deg = 1 for the identity dimension.
    s = 6
    mats = digital.sobol_matrices(s, sobol_direction_init(s, 0))
    polys = digital.primitive_polynomials(s - 1)
    deg = [1] + [p.bit_length() - 1 for p in polys]
    pts = digital.sobol_points(mats, 0, 1 << 12).astype(np.uint64)
    for a in range(s):
        for b in range(a + 1, s):
            t = net_t_value(pts[a], pts[b], 12)
            assert t <= (deg[a] - 1) + (deg[b] - 1), (a, b, t)


def test_one_dimensional_projections_are_01_sequences():
    mats = digital.sobol_matrices(8, sobol_direction_init(8, 0))
    pts = digital.sobol_points(mats, 0, 1 << 10).astype(np.uint64)
    for j in range(8):
        for m in range(11):
            n = 1 << m
            for b in range((1 << 10) // n):
                cells = pts[j, b * n:(b + 1) * n] >> np.uint64(32 - m) if m else np.zeros(1)
                assert np.unique(cells).size == n


def test_radical_inverse_digit_loop():
    i = np.array([0, 1, 2, 3, 6, 0xFFFFFFFF, 0x80000000], dtype=np.uint64)
    r = digital.radical_inverse_base2(i)
    assert list(map(int, r)) == [0, 1 << 31, 1 << 30, 3 << 30, 3 << 29, 0xFFFFFFFF, 1]
