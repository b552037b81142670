"""map_u32_to_unifloat, Sec. 2.1 (Floating Point Conversion) and Alg. 1.

The paper maps an integer u in [0, 2^32) to a float in [0, 1) that never reaches 1
and that is "optimal for 32 bits".  Its listing truncates: the result is the largest
IEEE binary32 value that does not exceed u * 2^-32.  That is the definition written
out here; the listing's leading-zero and bit-assembly construction is not used.
Zero maps to zero and one maps to 2^-32, the two special cases the listing spells out.
"""

import numpy as np

_TWO_M32 = 2.0 ** -32


def map_u32_to_unifloat(u):
    """Largest binary32 <= u / 2^32, elementwise (float32 array, same shape as u)."""
    u = np.asarray(u, dtype=np.uint64) & np.uint64(0xFFFFFFFF)
    exact = u.astype(np.float64) * _TWO_M32          # exact: u has at most 32 bits
    f = exact.astype(np.float32)                     # round to nearest even
    up = f.astype(np.float64) > exact                # rounded above the exact value?
    f = np.where(up, np.nextafter(f, np.float32(0)), f)
    return f.astype(np.float32)


def map_u32_to_unifloat_bits(u):
    """The binary32 bit pattern of map_u32_to_unifloat(u), as uint32."""
    return map_u32_to_unifloat(u).view(np.uint32)
