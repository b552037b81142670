"""Digital (t,s)-sequences in base 2: Sec. 2.2 (radical inversion), Sec. 2.3 (Eq. ts).

Conventions (the paper leaves them implicit):
  * An index i has binary digits a_k(i), k = 0 (least significant) upward.
  * A generator matrix C_j is stored as 32 columns of 32 bits; column k is the image
    of index digit a_k, and bit 31 of every column is the coefficient of 2^-1, bit 30
    of 2^-2, and so on.  The u32 result x represents x * 2^-32 in [0, 1).
  * Dimension 0 is the identity matrix (the van der Corput sequence, phi_2).
  * Dimensions j >= 1 are Sobol' matrices built from the (j-1)-th primitive
    polynomial over F_2, ordered by degree and then by the integer whose bits are
    the coefficients, with the classic Sobol' direction-number recurrence.
"""

import numpy as np

MASK32 = 0xFFFFFFFF


def radical_inverse_base2(i):
    """phi_2(i) * 2^32 for 0 <= i < 2^32: mirror the binary digits at the point (Sec. 2.2).

    Written as the digit loop of the definition, sum_k a_k(i) 2^(-k-1), scaled by 2^32.
    """
    i = np.asarray(i, dtype=np.uint64)
    out = np.zeros_like(i)
    for k in range(32):
        digit = (i >> np.uint64(k)) & np.uint64(1)
        out |= digit << np.uint64(31 - k)
    return out


def _gf2_mulmod(a, b, poly, deg):
    """a * b modulo poly over F_2 (polynomials as integers, bit t = coefficient of x^t)."""
    r = 0
    while b:
        if b & 1:
            r ^= a
        b >>= 1
        a <<= 1
        if a >> deg & 1:
            a ^= poly
    return r


def is_primitive(poly):
    """True iff poly (degree d >= 1, bit d set) is primitive over F_2.

    Brute force: the multiplicative order of x modulo poly must be exactly 2^d - 1.
    """
    deg = poly.bit_length() - 1
    if deg < 1:
        return False
    if deg == 1:
        return poly == 0b11          # x + 1 (the polynomial x is not primitive)
    if not poly & 1:
        return False                 # divisible by x
    period = (1 << deg) - 1
    x = 0b10
    acc = 1
    for k in range(1, period + 1):
        acc = _gf2_mulmod(acc, x, poly, deg)
        if acc == 1:
            return k == period
    return False


def primitive_polynomials(count):
    """The first `count` primitive polynomials over F_2, ordered by (degree, integer code)."""
    out = []
    deg = 1
    while len(out) < count:
        for code in range(1 << deg, 1 << (deg + 1)):
            if is_primitive(code):
                out.append(code)
                if len(out) == count:
                    break
        deg += 1
    return out


def direction_numbers(poly, m_init, nbits=32):
    """m_1..m_nbits for the Sobol' recurrence of primitive polynomial `poly`.

    With poly = x^d + a_1 x^(d-1) + ... + a_(d-1) x + 1 and m_1..m_d given (odd, m_k < 2^k):
      m_k = 2 a_1 m_(k-1) ^ 4 a_2 m_(k-2) ^ ... ^ 2^(d-1) a_(d-1) m_(k-d+1) ^ 2^d m_(k-d) ^ m_(k-d).
    """
    d = poly.bit_length() - 1
    m = [int(v) for v in m_init[:d]]
    for k in range(d, nbits):                       # computing m_(k+1), 0-based list index k
        v = m[k - d] ^ (m[k - d] << d)
        for r in range(1, d):
            if (poly >> (d - r)) & 1:
                v ^= m[k - r] << r
        m.append(v)
    return m[:nbits]


def generator_matrix_from_m(m):
    """32 columns (uint32) from direction numbers m_1..m_32: column k = m_(k+1) << (31-k)."""
    return np.array([(int(m[k]) << (31 - k)) & MASK32 for k in range(32)], dtype=np.uint32)


def identity_matrix():
    """Dimension 0: column k = 2^(31-k), i.e. x = phi_2(i) * 2^32 (van der Corput)."""
    return np.array([1 << (31 - k) for k in range(32)], dtype=np.uint32)


def sobol_matrices(s, direction_init):
    """Generator matrices for dims 0..s-1, uint32 [s][32].

    direction_init is [s][>=max degree] of initial m_k; row j is used for dimension j
    (row 0 is ignored: dimension 0 is the identity).
    """
    polys = primitive_polynomials(max(s - 1, 0))
    mats = np.zeros((s, 32), dtype=np.uint32)
    for j in range(s):
        if j == 0:
            mats[j] = identity_matrix()
        else:
            mats[j] = generator_matrix_from_m(direction_numbers(polys[j - 1], direction_init[j]))
    return mats


def digital_point(matrix, i):
    """x = XOR of the columns k with a_k(i) = 1 (Eq. ts over F_2), u32 as uint64 array."""
    i = np.asarray(i, dtype=np.uint64)
    x = np.zeros_like(i)
    for k in range(32):
        bit = (i >> np.uint64(k)) & np.uint64(1)
        x ^= np.where(bit == 1, np.uint64(int(matrix[k])), np.uint64(0))
    return x


def sobol_points(mats, first, n):
    """Unscrambled points x_i^(j) for i in [first, first+n), uint32 [s][n]."""
    idx = np.arange(n, dtype=np.uint64) + np.uint64(first)
    return np.stack([digital_point(mats[j], idx) for j in range(mats.shape[0])]).astype(np.uint32)
