"""Pins of the table-driven per-pixel XOR sampler (Sec. 2.6.1)."""

import numpy as np

from oracle import digital, estimator, scramble, xor_table
from synth import nus_seeds, sobol_direction_init, u32_draws


def _sobol_points(s, N, nus=False):
    mats = digital.sobol_matrices(s, sobol_direction_init(s, 0))
    pts = np.stack([digital.digital_point(mats[j], np.arange(N, dtype=np.uint64)) for j in range(s)])
    if nus:
        seeds = nus_seeds(s, 3)
        pts = np.stack([scramble.nested_uniform_scramble(pts[j], int(seeds[j])) for j in range(s)])
    return mats, pts.astype(np.uint32)


def _tables(s, N, seed):
    scr = u32_draws(seed, s * xor_table.CELLS).reshape(s, xor_table.CELLS)
    reo = (u32_draws(seed + 1, xor_table.CELLS) % np.uint32(N)).astype(np.uint32)
    return scr, reo


def test_brute_force_tiny():
    """Pixel by pixel, sample by sample, with the cell written out from (x, y)."""
    s, N, W, H = 3, 8, 130, 3
    _, pts = _sobol_points(s, N)
    scr, reo = _tables(s, N, 10)
    ps = np.repeat(np.arange(W * H), 2 * N)
    ii = np.tile(np.arange(2 * N), W * H)
    got = xor_table.xor_table_samples_u32(pts, scr, reo, W, ps, ii)
    k = 0
    for y in range(H):
        for x in range(W):
            c = (y % 128) * 128 + (x % 128)
            for i in range(2 * N):
                for j in range(s):
                    assert int(got[j, k]) == int(pts[j][(i ^ int(reo[c])) % N]) ^ int(scr[j][c]), (x, y, i, j)
                k += 1


def test_reordering_of_a_digital_net_is_a_digital_shift():
    """For unscrambled Sobol' points p_i = C i over F_2, so p_{i XOR r} = p_i XOR C r: sample i
    of a pixel is the i-th Sobol' point shifted by C r_c XOR s_c."""
    s, N, W = 4, 256, 300
    mats, pts = _sobol_points(s, N)
    scr, reo = _tables(s, N, 20)
    p = np.array([0, 1, 127, 128, 299, 300 * 5 + 7, 300 * 129 + 131], dtype=np.uint64)
    for pp in p:
        i = np.arange(N, dtype=np.uint64)
        got = xor_table.xor_table_samples_u32(pts, scr, reo, W, np.full(N, pp), i)
        y, x = divmod(int(pp), W)
        c = (y % 128) * 128 + x % 128
        for j in range(s):
            shift = int(digital.digital_point(mats[j], np.uint64(int(reo[c])))) ^ int(scr[j][c])
            want = scramble.shift_xor(digital.digital_point(mats[j], i), shift)
            assert np.array_equal(got[j], want.astype(np.uint32)), (pp, j)


def test_zero_tables_give_the_stored_points():
    s, N = 5, 64
    _, pts = _sobol_points(s, N, nus=True)
    zs, zr = np.zeros((s, xor_table.CELLS), np.uint32), np.zeros(xor_table.CELLS, np.uint32)
    i = np.arange(N)
    for pp in (0, 77, 5000):
        assert np.array_equal(xor_table.xor_table_samples_u32(pts, zs, zr, 200, np.full(N, pp), i), pts)


def test_tables_repeat_every_128_pixels_and_samples_every_N():
    s, N, W = 2, 32, 400
    _, pts = _sobol_points(s, N, nus=True)
    scr, reo = _tables(s, N, 30)
    i = np.arange(3 * N)
    f = lambda x, y: xor_table.xor_table_samples_u32(pts, scr, reo, W, np.full(i.size, y * W + x), i)
    a = f(5, 9)
    assert np.array_equal(a, f(5 + 128, 9)) and np.array_equal(a, f(5 + 256, 9 + 128))
    assert not np.array_equal(a, f(6, 9)) and not np.array_equal(a, f(5, 10))
    assert np.array_equal(a[:, :N], a[:, N:2 * N]) and np.array_equal(a[:, :N], a[:, 2 * N:])


def test_every_pixel_keeps_the_net_property():
    """Dims 0, 1 of N = 2^m scrambled Sobol' points form a (0, m, 2)-net; reindexing by XOR is
    a bijection of [0, N) and XOR of the digits a digital shift, so each pixel's first N
    samples are again a (0, m, 2)-net: every elementary box of volume 1/N holds one point."""
    m = 8
    N = 1 << m
    _, pts = _sobol_points(2, N, nus=True)
    scr, reo = _tables(2, N, 40)
    for pp in (0, 3, 129, 16383, 70000):
        got = xor_table.xor_table_samples_u32(pts, scr, reo, 1000, np.full(N, pp), np.arange(N))
        for a in range(m + 1):
            b = m - a
            keys = set(zip((got[0] >> np.uint32(32 - a)) if a else np.zeros(N, np.uint32),
                           (got[1] >> np.uint32(32 - b)) if b else np.zeros(N, np.uint32)))
            assert len(keys) == N, (pp, a)


def test_estimator_uses_the_table_sampler():
    s, N, W, H = 8, 128, 20, 6
    _, pts = _sobol_points(s, N, nus=True)
    scr, reo = _tables(s, N, 50)
    sp = {"kind": "xor_table", "s": s, "table": pts, "scramble": scr, "reorder": reo, "width": W}
    p, i = np.array([0, 7, 119]), np.array([5, 200, 127])
    assert np.array_equal(estimator.pixel_samples_u32(sp, p, i),
                          xor_table.xor_table_samples_u32(pts, scr, reo, W, p, i))
