"""Pins for the oracle's integer randomisation (Sec. 2.1, 2.3, 2.5.2).

The nested uniform scramble is builder-defined (the paper cites Owen scrambling
without fixing a function), so its values are not pinned; its defining properties are.
"""

import numpy as np

from oracle import digital, scramble
from synth import sobol_direction_init, u32_draws

from test_oracle_digital import net_t_value


def test_brev_is_an_involution_and_matches_string_reversal():
    x = u32_draws(20, 4096).astype(np.uint64)
    r = scramble.brev32(x)
    assert np.array_equal(scramble.brev32(r), x)
    for a, b in zip(x[:256], r[:256]):
        assert int(format(int(a), "032b")[::-1], 2) == int(b)


def test_nus_is_nested_bit_flip_structure():
    # Flipping the digit at MSB position k (bit 31-k) flips output digit k and leaves all
    # more significant output digits unchanged; the flip pattern below varies with the seed.
    x = u32_draws(21, 1 << 14).astype(np.uint64)
    s = u32_draws(22, 1 << 14).astype(np.uint64)
    y = scramble.nested_uniform_scramble(x, s)
    for k in range(32):
        bit = np.uint64(1 << (31 - k))
        y2 = scramble.nested_uniform_scramble(x ^ bit, s)
        d = y ^ y2
        above = ~np.uint64((1 << (32 - k)) - 1) & np.uint64(0xFFFFFFFF)
        assert np.all(d & bit)                 # its own digit always flips
        assert np.all((d & above) == 0)        # more significant digits never change
        if k < 24:
            # the next less significant digit flips in about half of the cases
            nxt = np.uint64(1 << (30 - k))
            frac = np.mean((d & nxt) != 0)
            assert 0.45 < frac < 0.55, (k, frac)


def test_nus_bijective_on_top16_domain():
    for seed in (0, 1, 0xDEADBEEF, 0xFFFFFFFF):
        h = np.arange(1 << 16, dtype=np.uint64) << np.uint64(16)
        y = scramble.nested_uniform_scramble(h, seed) >> np.uint64(16)
        assert np.unique(y).size == 1 << 16


def test_nus_digits_are_fair_across_seeds():
    # For a fixed input, each output digit is 1 for about half of the seeds.
    s = u32_draws(23, 1 << 14).astype(np.uint64)
    for xv in (0, 0x12345678, 0xFFFFFFFF):
        y = scramble.nested_uniform_scramble(np.full(s.size, xv, dtype=np.uint64), s)
        for k in range(24):
            frac = np.mean((y >> np.uint64(31 - k)) & np.uint64(1))
            assert 0.45 < frac < 0.55, (xv, k, frac)


def test_nus_and_xor_shift_preserve_02_nets():
    mats = digital.sobol_matrices(2, sobol_direction_init(2, 0))
    pts = digital.sobol_points(mats, 0, 1 << 16).astype(np.uint64)
    for seeds in ((1, 2), (0xA5A5A5A5, 0x5A5A5A5A)):
        x = scramble.nested_uniform_scramble(pts[0], seeds[0])
        y = scramble.nested_uniform_scramble(pts[1], seeds[1])
        xs = scramble.shift_xor(x, 0x9E3779B9)
        ys = scramble.shift_xor(y, 0x7F4A7C15)
        for m in range(17):
            n = 1 << m
            for b in range(min(4, (1 << 16) // n)):
                sl = slice(b * n, (b + 1) * n)
                assert net_t_value(x[sl], y[sl], m) == 0, (seeds, m, b)
                assert net_t_value(xs[sl], ys[sl], m) == 0, (seeds, m, b)


def test_scramble_changes_points():
    x = np.arange(1 << 10, dtype=np.uint64) << np.uint64(22)
    assert np.mean(scramble.nested_uniform_scramble(x, 7) != x) > 0.9


def test_shift_add_and_xor():
    assert int(scramble.shift_add(0xFFFFFFFF, 2)) == 1
    assert int(scramble.shift_xor(0xF0F0F0F0, 0xFFFF0000)) == 0x0F0FF0F0


def test_pixel_seed_derivation_varies_with_pixel_and_dimension():
    p = np.arange(4096, dtype=np.uint64)
    a = scramble.pixel_nus_seed(5, p, 0)
    b = scramble.pixel_nus_seed(5, p, 1)
    c = scramble.pixel_shift(5, p, 0)
    assert np.unique(a).size > 4090 and np.mean(a != b) > 0.99 and np.mean(a != c) > 0.99
