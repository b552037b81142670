"""64-bit indices and the partitioned enumeration of one sequence (Sec. 2.5.1; the 64-bit index
form of Alg. 3) — test infrastructure.

Indices are integers in [0, 2^64).

Wide generator matrices.  A Sobol' matrix with K columns (K <= 64) keeps, for column k, the
top 32 bits of the binary fraction m_(k+1) 2^-(k+1) of its direction number: m_(k+1) << (31-k)
for k < 32 and m_(k+1) >> (k-31) beyond (the rows stop at 2^-32, the precision of the u32
result).  Dimension 0 (the identity) has no digit below 2^-32 from index bits 32 and up, so
those columns are zero.  An index with a set bit at or above K is outside the matrix: the
calls refuse it instead of dropping the bit (Sec. 2.5.1 asks for certainty about the index
range).

Rank-1 lattice with a 64-bit index: floor(2^32 frac(phi_2(i) g)) with phi_2 over all 64
binary digits of i (Eq. R1LS).  Backward enumeration uses phi_2(2^64 - 1 - i).

Partition (Sec. 2.5.1).  The sequence is extended by one splitting dimension, the van der
Corput sequence phi_2(i); [0, 1) is cut into P = 2^q equal intervals and part p receives, in
index order, the indices i with floor(P phi_2(i)) = p.  The first q binary digits of phi_2(i)
are the q low bits of i in mirrored order, so part p holds exactly the indices with
i mod 2^q = rev_q(p): its m-th index is i = m 2^q + rev_q(p).  `part_indices_by_filter` is the
definition itself (a scan over all indices), kept for the tests that pin the enumeration.
"""

from fractions import Fraction

import numpy as np

from . import digital, scramble, unifloat

MASK32 = 0xFFFFFFFF
SHIFT_XOR = 1
LATTICE_BACKWARD = 2


def rev_bits(v, q):
    """The q low bits of v in mirrored order."""
    out = 0
    for k in range(q):
        out |= ((v >> k) & 1) << (q - 1 - k)
    return out


def phi2_64(i):
    """phi_2(i) for a 64-bit index, as an exact rational: sum_k a_k(i) 2^(-k-1)."""
    phi = Fraction(0)
    for k in range(64):
        if (i >> k) & 1:
            phi += Fraction(1, 1 << (k + 1))
    return phi


def part_index(q, p, m):
    """The m-th index of part p among 2^q parts (module docstring)."""
    return (m << q) | rev_bits(p, q)


def part_indices_by_filter(q, p, count):
    """The first `count` indices i with floor(2^q phi_2(i)) = p, by scanning i = 0, 1, ..."""
    out = []
    i = 0
    while len(out) < count:
        if int(phi2_64(i) * (1 << q)) == p:
            out.append(i)
        i += 1
    return out


def sobol_matrices_wide(s, direction_init, columns):
    """uint32 [s][columns] Sobol' matrices (dims 0..s-1, as digital.sobol_matrices) for
    indices below 2^columns."""
    assert 1 <= columns <= 64
    polys = digital.primitive_polynomials(max(s - 1, 0))
    mats = np.zeros((s, columns), dtype=np.uint32)
    for j in range(s):
        if j == 0:
            mats[j] = [(1 << (31 - k)) if k < 32 else 0 for k in range(columns)]
            continue
        m = digital.direction_numbers(polys[j - 1], direction_init[j], nbits=columns)
        for k in range(columns):
            v = m[k] << (31 - k) if k < 32 else m[k] >> (k - 31)
            mats[j, k] = v & MASK32
    return mats


def digital_point64(cols, i):
    """XOR of the columns k with bit k of i set (Eq. ts over F_2); i below 2^len(cols)."""
    i = int(i)
    assert i >> len(cols) == 0, "index outside the matrix"
    x = 0
    for k in range(len(cols)):
        if (i >> k) & 1:
            x ^= int(cols[k])
    return x


def lattice_point64(g, i, backward=False):
    """floor(2^32 frac(phi_2(i) g)) for a 64-bit index i.

    phi_2(i) = R / 2^64 with R the 64 digits of i mirrored, so frac(phi_2(i) g) 2^32 is
    (R g mod 2^64) / 2^32.
    """
    i = int(i)
    if backward:
        i = (1 << 64) - 1 - i
    r = rev_bits(i, 64)
    return ((r * int(g)) % (1 << 64)) >> 32


def _shift(v, delta, flags):
    if flags & SHIFT_XOR:
        return v ^ delta
    return (v + delta) & MASK32


def _indices(q, p, first, n):
    return [part_index(q, p, first + t) for t in range(n)]


def generate_sobol64(mats, q, p, first, n, nus_seeds=None, shifts=None, flags=0):
    """(u32 [s][n], f32 [s][n]): points first .. first+n-1 of part p of 2^q, dimension-major."""
    s = mats.shape[0]
    idx = _indices(q, p, first, n)
    out = np.zeros((s, n), dtype=np.uint32)
    for j in range(s):
        for t, i in enumerate(idx):
            out[j, t] = digital_point64(mats[j], i)
        if nus_seeds is not None:
            out[j] = scramble.nested_uniform_scramble(out[j].astype(np.uint64), int(nus_seeds[j])).astype(np.uint32)
        if shifts is not None:
            out[j] = [_shift(int(v), int(shifts[j]), flags) for v in out[j]]
    return out, unifloat.map_u32_to_unifloat(out)


def generate_lattice64(g, q, p, first, n, shifts=None, flags=0):
    """(u32 [s][n], f32 [s][n]) for the rank-1 lattice sequence, as generate_sobol64."""
    s = len(g)
    idx = _indices(q, p, first, n)
    out = np.zeros((s, n), dtype=np.uint32)
    for j in range(s):
        for t, i in enumerate(idx):
            v = lattice_point64(int(g[j]), i, backward=bool(flags & LATTICE_BACKWARD))
            out[j, t] = _shift(v, int(shifts[j]), flags) if shifts is not None else v
    return out, unifloat.map_u32_to_unifloat(out)
