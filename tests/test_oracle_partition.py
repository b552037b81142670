"""Pins of the oracle's 64-bit indices and partitioned enumeration (Sec. 2.5.1, Alg. 3's 64-bit
index form, Eq. R1LS with 64 binary digits)."""

from fractions import Fraction

import numpy as np
import pytest

from oracle import digital, lattice, partition
from synth import lattice_vector, sobol_direction_init, u32_draws


@pytest.mark.parametrize("q", [0, 1, 2, 3, 5])
def test_enumeration_is_the_interval_filter(q):
    """Part p's m-th index (closed form) = the m-th index whose phi_2 lies in [p/2^q, (p+1)/2^q)."""
    parts = range(1 << q) if q < 5 else (0, 7, 19, 31)
    for p in parts:
        want = partition.part_indices_by_filter(q, p, 24)
        got = [partition.part_index(q, p, m) for m in range(24)]
        assert got == want, (q, p)


def test_parts_tile_the_index_range():
    q, per = 4, 32
    seen = sorted(partition.part_index(q, p, m) for p in range(1 << q) for m in range(per))
    assert seen == list(range((1 << q) * per))


def test_rev_bits():
    assert partition.rev_bits(0b0011, 4) == 0b1100
    assert partition.rev_bits(1, 32) == 1 << 31
    assert partition.rev_bits(0, 0) == 0
    assert partition.rev_bits(0x12345678, 32) == int(digital.radical_inverse_base2(np.uint64(0x12345678)))


def test_phi2_64_definition():
    assert partition.phi2_64(1) == Fraction(1, 2)
    assert partition.phi2_64(6) == Fraction(3, 8)          # 110b -> 0.011b
    assert partition.phi2_64(1 << 63) == Fraction(1, 1 << 64)
    assert partition.phi2_64((1 << 64) - 1) == 1 - Fraction(1, 1 << 64)


def test_pascal_columns_beyond_32_follow_lucas():
    """Dimension 1 (x + 1) is the Pascal matrix: row r, column c is binom(c, r) mod 2, i.e. set
    iff r & c == r (Lucas), for every one of the 64 columns; row r is bit 31 - r."""
    init = sobol_direction_init(2, 0)
    mats = partition.sobol_matrices_wide(2, init, 64)
    for c in range(64):
        col = int(mats[1, c])
        for r in range(32):
            assert ((col >> (31 - r)) & 1) == int((r & c) == r), (r, c)


def test_identity_dimension_has_no_digit_from_high_index_bits():
    mats = partition.sobol_matrices_wide(1, sobol_direction_init(1, 0), 64)
    assert [int(v) for v in mats[0, :32]] == [1 << (31 - k) for k in range(32)]
    assert not mats[0, 32:].any()


def test_direction_numbers_odd_and_bounded_to_64():
    polys = digital.primitive_polynomials(31)
    init = sobol_direction_init(32, 0)
    for j, p in enumerate(polys, start=1):
        m = digital.direction_numbers(p, init[j], nbits=64)
        for k, v in enumerate(m, start=1):
            assert v & 1 and v < (1 << k), (p, k)


def test_wide_columns_are_the_top_32_bits_of_the_direction_fractions():
    """Column k holds floor(2^32 m_(k+1) / 2^(k+1)): the first 32 agree with the 32-column
    matrices, the rest are the same fractions truncated to 32 digits."""
    s = 8
    init = sobol_direction_init(s, 0)
    wide = partition.sobol_matrices_wide(s, init, 52)
    assert np.array_equal(wide[:, :32], digital.sobol_matrices(s, init))
    polys = digital.primitive_polynomials(s - 1)
    for j in range(1, s):
        m = digital.direction_numbers(polys[j - 1], init[j], nbits=52)
        for k in range(52):
            assert int(wide[j, k]) == int(Fraction(m[k], 1 << (k + 1)) * (1 << 32)), (j, k)


def test_digital_point64_below_2p32_and_linearity():
    mats = partition.sobol_matrices_wide(4, sobol_direction_init(4, 0), 64)
    rng = np.random.default_rng(1)
    for i in rng.integers(0, 2 ** 32, 50):
        for j in range(4):
            assert partition.digital_point64(mats[j], int(i)) == int(digital.digital_point(mats[j][:32], np.uint64(i)))
    for _ in range(50):
        a, b = (int(v) for v in rng.integers(0, 2 ** 63, 2, dtype=np.uint64))
        for j in range(4):
            assert partition.digital_point64(mats[j], a ^ b) == (partition.digital_point64(mats[j], a)
                                                                  ^ partition.digital_point64(mats[j], b))
    with pytest.raises(AssertionError):
        partition.digital_point64(mats[0][:40], 1 << 40)


def test_lattice64_is_the_rational_definition():
    rng = np.random.default_rng(2)
    for g in (1, 3, 0x9E3779B1, 0xFFFFFFFF):
        for i in list(rng.integers(0, 2 ** 63, 20, dtype=np.uint64)) + [0, 1, 2 ** 32, 2 ** 64 - 1]:
            i = int(i)
            x = partition.phi2_64(i) * g
            want = int((x - int(x)) * (1 << 32))
            assert partition.lattice_point64(g, i) == want, (g, i)
            xb = partition.phi2_64((1 << 64) - 1 - i) * g
            assert partition.lattice_point64(g, i, backward=True) == int((xb - int(xb)) * (1 << 32))


def test_lattice64_below_2p32_matches_the_32_bit_lattice():
    g = lattice_vector(6, 20, 3)
    idx = u32_draws(9, 200).astype(np.uint64)
    for j in range(6):
        want = lattice.lattice_point(int(g[j]), idx)
        got = [partition.lattice_point64(int(g[j]), int(i)) for i in idx]
        assert [int(v) for v in want] == got


def test_partitioned_lattice_is_the_shifted_scaled_subsequence():
    """phi_2(m 2^q + rev_q(p)) = (p + phi_2(m)) / 2^q, so the m-th point of part p is
    frac((p + phi_2(m)) g / 2^q)."""
    g = lattice_vector(3, 30, 5)
    for q, p in ((1, 1), (5, 19), (12, 3000), (32, 0xDEADBEEF)):
        for m in (0, 1, 2, 77, 2 ** 20 + 5, 2 ** 31 - 1):
            if m >> (64 - q):
                continue
            for j in range(3):
                x = (p + partition.phi2_64(m)) * int(g[j]) / (1 << q)
                want = int((x - int(x)) * (1 << 32))
                assert partition.lattice_point64(int(g[j]), partition.part_index(q, p, m)) == want


def test_splitting_dimension_selects_the_part():
    """The van der Corput values of part p's indices lie in [p/2^q, (p+1)/2^q)."""
    ident = partition.sobol_matrices_wide(1, sobol_direction_init(1, 0), 64)[0]
    for q, p in ((3, 5), (10, 777), (20, 12345)):
        for m in (0, 1, 9, 2 ** 33 + 17):
            x = partition.digital_point64(ident, partition.part_index(q, p, m))
            assert (x >> (32 - q)) == p


def test_subsequence_blocks_are_nets():
    """Sobol' dims 0..2 form a (1,3)-sequence, so dims (1, 2) of every part form (1, m, 2)-nets
    on aligned blocks of 2^m subsequence points (the block is a (1, m+q, 3)-net cut by an
    elementary interval of the splitting dimension)."""
    mats = partition.sobol_matrices_wide(3, sobol_direction_init(3, 0), 64)
    mexp, q, p = 8, 6, 37
    for m0 in (0, 1 << 40):
        pts = [[partition.digital_point64(mats[j], partition.part_index(q, p, m0 + t)) for t in range(1 << mexp)]
               for j in (1, 2)]
        for a in range(mexp):
            b = mexp - 1 - a           # volume 2^(1 - m): two points per box
            cells = {}
            for x, y in zip(*pts):
                key = (x >> (32 - a) if a else 0, y >> (32 - b) if b else 0)
                cells[key] = cells.get(key, 0) + 1
            assert len(cells) == 1 << (mexp - 1) and set(cells.values()) == {2}, (m0, a)


def test_generate_wrappers_shapes_and_shift():
    init = sobol_direction_init(3, 0)
    mats = partition.sobol_matrices_wide(3, init, 48)
    u, f = partition.generate_sobol64(mats, 4, 9, 1 << 40, 5, shifts=np.array([1, 2, 3], np.uint32))
    assert u.shape == (3, 5) and f.dtype == np.float32
    plain, _ = partition.generate_sobol64(mats, 4, 9, 1 << 40, 5)
    assert np.array_equal(u, (plain.astype(np.uint64) + np.array([[1], [2], [3]], np.uint64)).astype(np.uint32))
    ul, _ = partition.generate_lattice64(np.array([1, 3], np.uint32), 0, 0, 0, 4)
    assert [int(v) for v in ul[0]] == [0, 1 << 31, 1 << 30, 3 << 30]
