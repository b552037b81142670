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


def _lattice_sampler(s, W, table, flags=estimator.PIXEL_SHIFT | estimator.PIXEL_TABLE_SHIFT):
    from synth import lattice_vector

    g = lattice_vector(s, 20, 3)
    return g, {"kind": "lattice", "s": s, "table": g, "seed": 0, "flags": flags, "width": W, "height": 4,
               "shift_table": table}


def test_constant_shift_table_is_a_global_rotation():
    """All cells holding (a, b): the lattice rotated by (a, b, a, b, ...) (the generator's own
    rotation path); with XOR, the digital shift."""
    from oracle import generate

    s, W, n = 5, 300, 64
    a, b = 0x9E3779B9, 0x12345678
    table = np.stack([np.full(xor_table.CELLS, a, np.uint32), np.full(xor_table.CELLS, b, np.uint32)])
    for xor in (0, estimator.SHIFT_XOR):
        g, sp = _lattice_sampler(s, W, table, estimator.PIXEL_SHIFT | estimator.PIXEL_TABLE_SHIFT | xor)
        want, _ = generate.generate_lattice(g, 0, n, np.array([a, b, a, b, a], np.uint32), xor)
        for pp in (0, 1000):
            got = estimator.pixel_samples_u32(sp, np.full(n, pp), np.arange(n))
            assert np.array_equal(got, want), (xor, pp)


def test_shift_table_pairs_of_dimensions_and_tiling():
    s, W, n = 6, 400, 32
    table = u32_draws(60, 2 * xor_table.CELLS).reshape(2, xor_table.CELLS)
    g, sp = _lattice_sampler(s, W, table)
    _, plain = _lattice_sampler(s, W, table, 0)
    i = np.arange(n)
    f = lambda x, y: estimator.pixel_samples_u32(sp, np.full(n, y * W + x), i).astype(np.uint64)
    base = estimator.pixel_samples_u32(plain, np.zeros(n, np.int64), i).astype(np.uint64)
    a = f(7, 3)
    d = (a - base) & np.uint64(0xFFFFFFFF)       # the rotation of each component
    assert all(len(set(d[j].tolist())) == 1 for j in range(s))
    assert d[0, 0] == d[2, 0] == d[4, 0] and d[1, 0] == d[3, 0] == d[5, 0]
    assert d[0, 0] == table[0][3 * 128 + 7] and d[1, 0] == table[1][3 * 128 + 7]
    assert np.array_equal(a, f(7 + 128, 3 + 256)) and not np.array_equal(a, f(8, 3))


def test_rotated_lattice_keeps_one_point_per_interval():
    """A rotated rank-1 lattice with odd generator components: each pixel's first 2^m points have
    one coordinate in every interval [k/2^m, (k+1)/2^m) in every dimension."""
    s, W, m = 4, 200, 7
    table = u32_draws(61, 2 * xor_table.CELLS).reshape(2, xor_table.CELLS)
    _, sp = _lattice_sampler(s, W, table)
    for pp in (0, 129, 4321):
        got = estimator.pixel_samples_u32(sp, np.full(1 << m, pp), np.arange(1 << m))
        for j in range(s):
            assert len(set((got[j] >> np.uint32(32 - m)).tolist())) == 1 << m, (pp, j)
