"""Per-pixel rank-1 lattice samplers of Sec. 2.4 and Sec. 3 (test infrastructure only).

Two ways of giving every pixel its own copy of a rank-1 lattice sequence:

* random generator vector (Alg. 4): component j of pixel p uses g_pj = hash | 1, the hash
  depending on (j, pixel).  The paper leaves the hash open.  Reading: the same chained hash as
  the per-pixel scramble seeds, k_pj = H(H(seed + 2j) ^ p), and g_pjc = H(k_pj + c) | 1 for
  instance c.  With four instances superimposed, sample i of the pixel belongs to instance
  c = i mod 4 and is point floor(i / 4) of that instance's sequence.
* pixel-shifted lattice (Eq. PixelShiftedR1LS): one shift per pixel, added to the radical
  inverse before the multiplication by the shared generator vector,
      x_i^(j) = (phi_2(i) + phi_3(h(x, y))) g_j  mod 1,
  with h(x, y) the index of pixel (x, y) along the Hilbert curve over the image plane.
  Readings: in 32-bit fixed point the shift is floor(2^32 phi_3(h)); the curve covers the
  2^k x 2^k square with 2^k >= max(width, height), starts in cell (0, 0), and visits the four
  quadrants of a square in the order (0,0), (0,1), (1,1), (1,0) (x = column, y = row), the two
  quadrants with y < half with the sub-curve transposed, the one with x >= half about the other
  diagonal, so that consecutive indices are edge-adjacent cells.

Everything is exact integer arithmetic; H is the hash of `scramble.pcg_hash`.
"""

from fractions import Fraction

import numpy as np

from .digital import radical_inverse_base2
from .scramble import pcg_hash

_M = 0xFFFFFFFF


def radical_inverse_u32(n, base):
    """floor(2^32 * phi_b(n)) for a non-negative integer n: phi_b mirrors the base-b digits of
    n at the radix point (Sec. 2.2), evaluated exactly with rationals."""
    n = int(n)
    phi = Fraction(0)
    scale = Fraction(1, base)
    while n:
        n, digit = divmod(n, base)
        phi += digit * scale
        scale /= base
    return int(phi * (1 << 32))  # floor: phi >= 0


def hilbert_order(width, height):
    """Smallest k with 2^k >= max(width, height) (k >= 1)."""
    k = 1
    while (1 << k) < max(width, height):
        k += 1
    return k


def hilbert_index(x, y, order):
    """Position of cell (x, y) along the Hilbert curve of the 2^order square (module docstring)."""
    if order == 0:
        return 0
    half = 1 << (order - 1)
    qx, qy = int(x >= half), int(y >= half)
    xl, yl = x - half * qx, y - half * qy
    quadrant = {(0, 0): 0, (0, 1): 1, (1, 1): 2, (1, 0): 3}[(qx, qy)]
    if qy == 0:
        if qx == 0:
            xl, yl = yl, xl  # transposed sub-curve
        else:
            xl, yl = half - 1 - yl, half - 1 - xl  # transposed about the other diagonal
    return quadrant * half * half + hilbert_index(xl, yl, order - 1)


def pixel_hilbert_shift(p, width, height):
    """floor(2^32 phi_3(h(x, y))) for pixel p = y * width + x."""
    p = int(p)
    return radical_inverse_u32(hilbert_index(p % width, p // width, hilbert_order(width, height)), 3)


def pixel_generator(seed, p, j, c=0):
    """g_pjc = H(H(H(seed + 2j) ^ p) + c) | 1, odd (Alg. 4 with the hash reading above)."""
    k = pcg_hash(pcg_hash((int(seed) + 2 * int(j)) & _M) ^ (int(p) & _M))
    return pcg_hash((k + int(c)) & _M) | 1


def pixel_lattice_points(g, i, shift=0, backward=False):
    """(phi_2(i') + shift) g mod 1 as u32 for index array i (i' = 2^32 - 1 - i when backward)."""
    i = np.asarray(i, dtype=np.uint64)
    if backward:
        i = np.uint64(_M) - i
    r = (radical_inverse_base2(i) + np.uint64(int(shift) & _M)) & np.uint64(_M)
    return (r * np.uint64(int(g) & _M)) & np.uint64(_M)
