"""Pins for the oracle's per-pixel hash, the "pcg" hash of Jarzynski and Olano (JCGT 9(3),
2020): a PCG state step (a full-period linear congruential generator mod 2^32) followed by the
RXS-M-XS output permutation.  It feeds the per-pixel randomisation of Sec. 2.5.2 and the
per-pixel generator of Alg. 4.

No output values of the published hash are available offline, so its values stay "parity
unpinned"; what is pinned here is its structure.  Every stage is a bijection of the 32-bit
words, so the hash is one too, and each stage has an inverse that follows from its definition
alone (written below without any code of the oracle):
  * the LCG step v -> a v + c is undone with the multiplicative inverse of the odd a mod 2^32;
  * the random xorshift x -> x ^ (x >> (4 + top4(x))) leaves the top 4 bits unchanged (the shift
    is at least 4), so the shift can be read from the result and the xorshift undone by
    repeated substitution;
  * the multiply by the odd m is undone with m^-1 mod 2^32;
  * the final xorshift by 22 >= 16 is its own inverse.
A slip in the oracle (a dropped "+ 4", an even or mistyped multiplier, another shift) breaks
the round trip; the last test plants such slips in copies of the hash and checks that the
round trip catches each of them.
"""

import numpy as np
import pytest

from oracle import scramble
from synth import u32_draws

M32 = 1 << 32

# Published constants of the hash: PCG's 32-bit LCG multiplier and increment, and the RXS-M-XS
# output multiplier.
LCG_A = 747796405
LCG_C = 2891336453
RXS_M = 277803737


def _inv_mod_2_32(a):
    """Multiplicative inverse of an odd a modulo 2^32 by Newton's iteration x <- x (2 - a x),
    which doubles the number of correct low bits each step (a x = 1 mod 8 for x = a)."""
    assert a & 1
    x = a
    for _ in range(5):
        x = (x * (2 - a * x)) % M32
    return x


def _undo_xorshift_right(y, r):
    """x with x ^ (x >> r) == y (x = y ^ (x >> r), iterated until every bit is settled)."""
    x = y
    for _ in range(32 // r + 1):
        x = y ^ (x >> r)
    return x


def inverse_pcg(h):
    """The preimage of h under the hash, derived stage by stage from the definition."""
    h = int(h)
    word = _undo_xorshift_right(h, 22)
    rxs = (word * _inv_mod_2_32(RXS_M)) % M32
    shift = (rxs >> 28) + 4
    state = _undo_xorshift_right(rxs, shift)
    return ((state - LCG_C) * _inv_mod_2_32(LCG_A)) % M32


def test_constants_give_a_full_period_generator_and_invertible_multiplier():
    # Hull-Dobell: x -> a x + c mod 2^32 has period 2^32 iff c is odd and a = 1 mod 4.
    assert LCG_C % 2 == 1 and LCG_A % 4 == 1
    assert RXS_M % 2 == 1
    for a in (LCG_A, RXS_M, 3, 0xFFFFFFFF):
        assert (a * _inv_mod_2_32(a)) % M32 == 1
        assert pow(a, -1, M32) == _inv_mod_2_32(a)


def test_inverse_pcg_undoes_the_hash_on_seeded_and_edge_inputs():
    x = u32_draws(31, 1 << 20).astype(np.uint64)
    edges = np.array([0, 1, 2, 3, 0x7FFFFFFF, 0x80000000, 0xFFFFFFFE, 0xFFFFFFFF, LCG_C, (M32 - LCG_C) % M32,
                      0x0FFFFFFF, 0xF0000000], dtype=np.uint64)
    x = np.concatenate([edges, x])
    h = scramble.pcg_hash(x)
    assert h.dtype == np.uint64 and int(h.max()) < M32
    inv = np.frompyfunc(inverse_pcg, 1, 1)
    back = inv(h).astype(np.uint64)
    bad = np.nonzero(back != x)[0]
    assert bad.size == 0, (x[bad[:5]], h[bad[:5]], back[bad[:5]])


def test_every_shift_amount_of_the_random_xorshift_is_exercised():
    # The RXS shift is 4 + the top 4 bits of the LCG state: all 16 amounts occur among the
    # seeded inputs, so the round trip above covers each branch of the inversion.
    x = u32_draws(32, 1 << 12).astype(np.uint64)
    state = (x * np.uint64(LCG_A) + np.uint64(LCG_C)) & np.uint64(M32 - 1)
    assert np.unique(state >> np.uint64(28)).size == 16


def test_hash_is_a_bijection_on_a_block_of_inputs():
    # 2^20 consecutive inputs give 2^20 distinct outputs (a consequence of the inverse).
    x = np.arange(1 << 20, dtype=np.uint64) + np.uint64(0x9E3779B9)
    assert np.unique(scramble.pcg_hash(x)).size == 1 << 20


def _mutant(kind):
    """Copies of the hash with one plausible slip each (planted on the CPU, in test code)."""
    m = np.uint64(M32 - 1)

    def h(v):
        v = np.asarray(v, dtype=np.uint64) & m
        a = np.uint64(LCG_A + 2 if kind == "lcg_a" else LCG_A)
        c = np.uint64(LCG_C - 1 if kind == "lcg_c" else LCG_C)
        state = (v * a + c) & m
        add = np.uint64(0 if kind == "no_plus4" else 4)
        shift = (state >> np.uint64(28)) + add
        word = (state >> shift) ^ state
        mult = np.uint64(RXS_M + 1 if kind == "even_mult" else RXS_M)
        word = (word * mult) & m
        fs = np.uint64(21 if kind == "final_shift" else 22)
        return ((word >> fs) ^ word) & m

    return h


@pytest.mark.parametrize("kind", ["no_plus4", "even_mult", "lcg_a", "lcg_c", "final_shift"])
def test_round_trip_catches_planted_slips(kind):
    x = u32_draws(33, 4096).astype(np.uint64)
    h = _mutant(kind)(x)
    back = np.array([inverse_pcg(int(v)) for v in h], dtype=np.uint64)
    assert np.any(back != x), kind
    # and the unmutated copy passes the same check
    h0 = _mutant("none")(x)
    assert np.array_equal(h0, scramble.pcg_hash(x))
