"""The table-driven per-pixel samplers of Sec. 2.6.1 (image-plane decorrelation) — test
infrastructure.

One set of N stored s-dimensional integer points P = (p_0, ..., p_{N-1}) (in the paper,
Owen-scrambled Sobol' points) serves every pixel.  Two tables, indexed by the pixel's
position modulo a 128 x 128 tile, c = (y mod 128) * 128 + (x mod 128), randomise it per
pixel: a reordering integer r_c (128^2 entries) and a digit scramble s_{c,j} (128^2 x s
entries).  Sample i of the pixel at (x, y), dimension j, is the stored point with index
i XOR r_c, its digits XORed with s_{c,j}; the integer is then mapped to [0, 1) as every other
sample (Sec. 2.1).

Reading (the paper states the rule for indices inside the stored set only): N is a power of
two and the index i XOR r_c is taken modulo N, so the stored points repeat with period N and
an r_c >= N acts through its low bits.  For i < N and r_c < N the reduction changes nothing.

The tables themselves (found by simulated annealing in the paper) are inputs; any tables of
the right shape give a valid sampler.

Table of rotations.  The second sampler of the section keeps the sequence (a rank-1 lattice
sequence in the paper) and rotates it per pixel by a two-dimensional shift read from one
128 x 128 table, the same vector for every pair of dimensions: component j of the pixel in
cell c is rotated by t_{c, j mod 2} (integer rotation mod 2^32, or XOR), in place of the
hashed per-pixel rotation.
"""

import numpy as np

from . import unifloat

TILE = 128
CELLS = TILE * TILE


def pixel_cell(p, width):
    """c = (y mod 128) * 128 + (x mod 128) for pixel p = y * width + x."""
    p = np.asarray(p, dtype=np.uint64)
    y = p // np.uint64(width)
    x = p - y * np.uint64(width)
    return (y % np.uint64(TILE)) * np.uint64(TILE) + (x % np.uint64(TILE))


def xor_table_samples_u32(points, scramble_table, reorder, width, p, i):
    """uint32 [s][n]: sample i[k] of pixel p[k], every dimension of `points` (uint32 [s][N])."""
    points = np.asarray(points, dtype=np.uint32)
    s, N = points.shape
    assert N > 0 and N & (N - 1) == 0, "the number of stored points must be a power of two"
    c = pixel_cell(p, width)
    idx = (np.asarray(i, dtype=np.uint64) ^ np.asarray(reorder, dtype=np.uint64)[c]) % np.uint64(N)
    out = np.zeros((s, idx.size), dtype=np.uint32)
    for j in range(s):
        out[j] = points[j][idx] ^ np.asarray(scramble_table, dtype=np.uint32)[j][c]
    return out


def xor_table_samples_f32(points, scramble_table, reorder, width, p, i):
    return unifloat.map_u32_to_unifloat(xor_table_samples_u32(points, scramble_table, reorder, width, p, i))


def table_shift(shift_table, width, p, j):
    """The rotation of component j for pixels p: entry j mod 2 of the cell's shift vector;
    shift_table is uint32 [2][128^2]."""
    return np.asarray(shift_table, dtype=np.uint64)[j % 2][pixel_cell(p, width)]
