"""Randomisation kept in integers: Sec. 2.1 (scrambling and Cranley-Patterson rotation
computed on integers before conversion), Sec. 2.3 (digit scrambling by XOR) and
Sec. 2.5.2 (one independent randomisation per processing element).

Nested uniform scramble.  The paper cites Owen scrambling (Sec. 2.1, 2.5.2, 2.6.1) but
defines no scramble function, so this library defines one.  A nested uniform scramble
of a 32-bit binary fraction must flip each digit by a pseudo-random function of the
seed and of all digits that are *more* significant.  After mirroring the bits, more
significant digits become lower bits, and any composition of the operations below only
carries information from lower to higher bits, so it has exactly that structure:

  NUS_s(x) = brev( P_s( brev(x) ) ), with P_s(v) (all arithmetic mod 2^32, lo24 = v & 0xFFFFFF):
    v = v + s
    v = v + lo24(v) * 0x612362
    v = v ^ (v << 8)
    v = v + lo24(v) * ((s >> 8) & 0xFFFFFE)
    v = v + lo24(v) * 0x934C76
    v = v ^ (v << 9)
    v = v ^ (v * 0xFA8F38AA)

Every multiplier is even, so product bit k depends only on bits below k.  The constants
were chosen by an avalanche search (flip probabilities within noise of 1/2 for all bit
pairs of the 24 most significant digits).

Shift: y + delta mod 2^32 (integer Cranley-Patterson rotation, default) or y ^ delta
(digital shift).

Per-pixel seeds use the hash "pcg" of Jarzynski and Olano, "Hash Functions for GPU
Rendering", JCGT 9(3), 2020 (a permuted congruential step followed by an RXS-M-XS output
permutation), written here from that definition:
  state = v * 747796405 + 2891336453
  word  = ((state >> ((state >> 28) + 4)) ^ state) * 277803737
  hash  = (word >> 22) ^ word
"""

import numpy as np

from .digital import radical_inverse_base2

_M = np.uint64(0xFFFFFFFF)
_LO24 = np.uint64(0xFFFFFF)


def _u(x):
    return np.asarray(x, dtype=np.uint64) & _M


def brev32(x):
    """Mirror the 32 bits of x (bit k moves to bit 31-k): phi_2 on the integer grid."""
    return radical_inverse_base2(_u(x))


def nus_permute(v, s):
    """P_s: the low-to-high mixing applied to the mirrored value (see module docstring)."""
    v = _u(v)
    s = _u(s)
    v = (v + s) & _M
    v = (v + (v & _LO24) * np.uint64(0x612362)) & _M
    v = v ^ ((v << np.uint64(8)) & _M)
    v = (v + (v & _LO24) * ((s >> np.uint64(8)) & np.uint64(0xFFFFFE))) & _M
    v = (v + (v & _LO24) * np.uint64(0x934C76)) & _M
    v = v ^ ((v << np.uint64(9)) & _M)
    v = v ^ ((v * np.uint64(0xFA8F38AA)) & _M)
    return v


def nested_uniform_scramble(x, seed):
    """NUS_seed(x) for 32-bit x (vectorised; seed broadcasts)."""
    return brev32(nus_permute(brev32(x), seed))


def shift_add(y, delta):
    """Integer Cranley-Patterson rotation: (y + delta) mod 2^32."""
    return (_u(y) + _u(delta)) & _M


def shift_xor(y, delta):
    """Digital shift: y XOR delta."""
    return _u(y) ^ _u(delta)


def pcg_hash(v):
    """The 'pcg' integer hash (Jarzynski and Olano 2020), vectorised, on uint64-held u32."""
    v = _u(v)
    state = (v * np.uint64(747796405) + np.uint64(2891336453)) & _M
    shift = (state >> np.uint64(28)) + np.uint64(4)
    word = (((state >> shift) ^ state) * np.uint64(277803737)) & _M
    return ((word >> np.uint64(22)) ^ word) & _M


def dim_key(seed, slot):
    """Per-dimension key H(seed + slot) (slot = 2j for scramble seeds, 2j+1 for shifts)."""
    return pcg_hash((_u(seed) + _u(slot)) & _M)


def pixel_nus_seed(seed, p, j):
    """Scramble seed of dimension j in pixel p: H(H(seed + 2j) ^ p)."""
    return pcg_hash(dim_key(seed, 2 * np.asarray(j, dtype=np.uint64)) ^ _u(p))


def pixel_shift(seed, p, j):
    """Shift of dimension j in pixel p: H(H(seed + 2j + 1) ^ p)."""
    return pcg_hash(dim_key(seed, 2 * np.asarray(j, dtype=np.uint64) + 1) ^ _u(p))


def pixel_offset_u32(pixel_seed, p, j):
    """Raw 32 bits behind the per-pixel integrand offset: H(H(pixel_seed + j) ^ p)."""
    return pcg_hash(pcg_hash((_u(pixel_seed) + _u(j)) & _M) ^ _u(p))
