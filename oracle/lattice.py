"""Rank-1 lattice sequences in base 2: Sec. 2.4, Eq. (R1LS), Alg. 4.

x_i^(j) = (phi_2(i) * g_j) mod 1.  With phi_2(i) = r / 2^32 for the mirrored integer r,
(r * g_j mod 2^32) / 2^32 is that point exactly: dropping the high word of the 32x32-bit
product is the "mod 1" (Alg. 4 caption).  Backward enumeration (Alg. 4) uses phi_2 of
2^32 - 1 - i, so that the origin comes last instead of first.
"""

import numpy as np

from .digital import radical_inverse_base2

_M = np.uint64(0xFFFFFFFF)


def lattice_points(g, first, n, backward=False):
    """Unshifted lattice points for i in [first, first+n), uint32 [s][n]."""
    idx = np.arange(n, dtype=np.uint64) + np.uint64(first)
    if backward:
        idx = np.uint64(0xFFFFFFFF) - idx
    r = radical_inverse_base2(idx)
    g = np.asarray(g, dtype=np.uint64)
    return ((r[None, :] * g[:, None]) & _M).astype(np.uint32)


def lattice_point(g_j, i, backward=False):
    """One component (phi_2(i) * g_j mod 1) * 2^32 for index array i."""
    i = np.asarray(i, dtype=np.uint64)
    if backward:
        i = np.uint64(0xFFFFFFFF) - i
    return (radical_inverse_base2(i) * np.uint64(int(g_j))) & _M
