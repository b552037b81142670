"""Pins of the oracle's per-pixel lattice samplers (Alg. 4; Eq. PixelShiftedR1LS; Sec. 2.2)."""

import itertools
from fractions import Fraction

import numpy as np
import pytest

from oracle import digital, estimator, lattice, pixel_lattice as pl, scramble
from synth import lattice_vector


def test_radical_inverse_base3_closed_forms():
    # phi_3(1) = 1/3, phi_3(2) = 2/3, phi_3(3) = 1/9, phi_3(4) = 1/9 + 1/3, phi_3(5) = 1/9 + 2/3
    for n, q in ((0, Fraction(0)), (1, Fraction(1, 3)), (2, Fraction(2, 3)), (3, Fraction(1, 9)),
                 (4, Fraction(4, 9)), (5, Fraction(7, 9)), (9, Fraction(1, 27)), (26, Fraction(26, 27))):
        assert pl.radical_inverse_u32(n, 3) == (q.numerator << 32) // q.denominator


def test_radical_inverse_base3_is_a_permutation_of_the_grid():
    m = 6
    got = sorted(pl.radical_inverse_u32(n, 3) for n in range(3 ** m))
    assert got == [(k << 32) // 3 ** m for k in range(3 ** m)]


def test_radical_inverse_base2_is_bit_reversal():
    rng = np.random.default_rng(0)
    for n in rng.integers(0, 2 ** 32, 200):
        assert pl.radical_inverse_u32(int(n), 2) == int(scramble.brev32(np.uint64(n)))


def test_hilbert_order_one_and_endpoints():
    # cells (x, y) visited in the order (0,0), (0,1), (1,1), (1,0)
    assert [pl.hilbert_index(x, y, 1) for x, y in ((0, 0), (0, 1), (1, 1), (1, 0))] == [0, 1, 2, 3]
    for k in range(1, 7):
        n = 1 << k
        assert pl.hilbert_index(0, 0, k) == 0
        assert pl.hilbert_index(n - 1, 0, k) == n * n - 1


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6])
def test_hilbert_is_a_continuous_bijection(k):
    n = 1 << k
    cell = {}
    for x, y in itertools.product(range(n), range(n)):
        cell[pl.hilbert_index(x, y, k)] = (x, y)
    assert sorted(cell) == list(range(n * n))
    for d in range(n * n - 1):
        (x0, y0), (x1, y1) = cell[d], cell[d + 1]
        assert abs(x0 - x1) + abs(y0 - y1) == 1, d


def test_hilbert_quadrants_hold_consecutive_blocks():
    k = 5
    q = 1 << (k - 1)
    for (qx, qy), block in (((0, 0), 0), ((0, 1), 1), ((1, 1), 2), ((1, 0), 3)):
        vals = {pl.hilbert_index(qx * q + x, qy * q + y, k) for x in range(q) for y in range(q)}
        assert vals == set(range(block * q * q, (block + 1) * q * q))


def test_hilbert_order_of_image_sizes():
    assert pl.hilbert_order(1920, 1080) == 11
    assert pl.hilbert_order(3840, 2160) == 12
    assert pl.hilbert_order(2, 1) == 1
    assert pl.hilbert_order(1024, 3) == 10


def test_pixel_generator_is_odd_and_varies():
    gs = {pl.pixel_generator(7, p, j, c) for p in range(40) for j in range(3) for c in range(4)}
    assert all(g & 1 for g in gs)
    assert len(gs) == 40 * 3 * 4  # distinct draws (collisions would be a 1e-6 event)


def test_pixel_shift_is_a_rotation_of_the_lattice():
    """(phi_2(i) + s) g = phi_2(i) g + s g (mod 1): the shifted sequence is the lattice
    sequence rotated by s g, which for i < 2^m is the shifted lattice {k g / 2^m + s g}."""
    g = int(lattice_vector(1, 20, 3)[0])
    s = pl.pixel_hilbert_shift(12345, 1920, 1080)
    i = np.arange(1 << 10, dtype=np.uint64)
    for back in (False, True):
        got = pl.pixel_lattice_points(g, i, s, back)
        want = (lattice.lattice_point(g, i, backward=back) + np.uint64((s * g) & 0xFFFFFFFF)) & np.uint64(0xFFFFFFFF)
        assert np.array_equal(got, want)
    m = 10
    pts = pl.pixel_lattice_points(g, i, s) >> np.uint64(32 - m)  # top m bits: the lattice cell
    assert sorted(pts.tolist()) == list(range(1 << m))  # one point per 2^-m interval (g odd)


def test_estimator_options_compose_as_defined():
    """Sampler flags of the per-pixel lattice: each option against the definition."""
    W, H = 13, 5
    s = 3
    g = lattice_vector(s, 20, 3)
    base = {"kind": "lattice", "s": s, "table": g, "seed": 99, "width": W, "height": H}
    p = np.repeat(np.arange(W * H, dtype=np.uint64), 12)
    i = np.tile(np.arange(12, dtype=np.uint64), W * H)
    plain = estimator.pixel_samples_u32(dict(base, flags=0), p, i)
    assert np.array_equal(plain, lattice.lattice_points(g, 0, 12).repeat(1, axis=1)[:, np.tile(np.arange(12), W * H)])
    hil = estimator.pixel_samples_u32(dict(base, flags=estimator.PIXEL_HILBERT_SHIFT), p, i)
    for k in (0, 17, 64):
        pp = int(p[k * 12])
        sh = pl.pixel_hilbert_shift(pp, W, H)
        for j in range(s):
            want = pl.pixel_lattice_points(int(g[j]), np.arange(12, dtype=np.uint64), sh)
            assert np.array_equal(hil[j, k * 12:(k + 1) * 12], want.astype(np.uint32))
    rnd = estimator.pixel_samples_u32(dict(base, flags=estimator.PIXEL_RANDOM_GENERATOR | estimator.LATTICE_INSTANCES4
                                           | estimator.LATTICE_BACKWARD), p, i)
    pp = 7
    for j in range(s):
        for n in range(12):
            c, ii = n % 4, n // 4
            gg = pl.pixel_generator(99, pp, j, c)
            want = (int(scramble.brev32(np.uint64(0xFFFFFFFF - ii))) * gg) & 0xFFFFFFFF
            assert int(rnd[j, pp * 12 + n]) == want


def test_hilbert_shifts_of_neighbouring_pixels_differ():
    W, H = 64, 64
    shifts = {pl.pixel_hilbert_shift(p, W, H) for p in range(W * H)}
    assert len(shifts) == W * H  # phi_3 of distinct indices are distinct
