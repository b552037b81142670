"""Pins for the oracle's map_u32_to_unifloat (Sec. 2.1, Alg. 1)."""

import os
import struct
from fractions import Fraction

import numpy as np

from oracle.unifloat import map_u32_to_unifloat, map_u32_to_unifloat_bits
from synth import u32_draws

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "unifloat_listing.txt")


def _listing_construction(u):
    """The paper's bit assembly (exponent 126 - clz, truncated mantissa), on Python ints."""
    if u == 0:
        return 0
    if u == 1:
        return (126 - 31) << 23
    z = 32 - u.bit_length()
    e = 126 - z
    m = ((u << (z + 1)) & 0xFFFFFFFF) >> 9
    return (e << 23) | m


def _f32(bits):
    return struct.unpack("<f", struct.pack("<I", bits))[0]


def test_listing_values():
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        u, bits = (int(t, 16) for t in line.split())
        assert int(map_u32_to_unifloat_bits(np.array([u]))[0]) == bits, hex(u)


def test_matches_listing_construction_on_random_and_edge_inputs():
    u = u32_draws(11, 1 << 20).astype(np.uint64)
    edges = []
    for k in range(32):
        for d in (-2, -1, 0, 1, 2):
            v = (1 << k) + d
            if 0 <= v < 1 << 32:
                edges.append(v)
    u = np.concatenate([u, np.array(edges + [0xFFFFFFFF, 0xFFFFFFFE], dtype=np.uint64)])
    got = map_u32_to_unifloat_bits(u)
    want = np.array([_listing_construction(int(v)) for v in u], dtype=np.uint64)
    assert np.array_equal(got.astype(np.uint64), want)


def test_largest_float_not_above_exact_value():
    # Exact rational check: f <= u / 2^32 < next float above f.
    u = u32_draws(12, 2000).astype(np.uint64)
    bits = map_u32_to_unifloat_bits(u)
    for ui, b in zip(u, bits):
        f = Fraction(_f32(int(b)))
        nxt = Fraction(_f32(int(b) + 1))
        exact = Fraction(int(ui), 1 << 32)
        assert f <= exact < nxt


def test_never_reaches_one_and_monotone():
    u = np.sort(u32_draws(13, 1 << 18).astype(np.uint64))
    f = map_u32_to_unifloat(u)
    assert np.all(f < 1.0)
    assert np.all(np.diff(f.astype(np.float64)) >= 0)
    assert map_u32_to_unifloat(np.array([0xFFFFFFFF]))[0] < 1.0


def test_exact_and_injective_below_2_24():
    u = np.arange(1 << 24, dtype=np.uint64)
    f = map_u32_to_unifloat(u).astype(np.float64)
    assert np.array_equal(f, u.astype(np.float64) * 2.0 ** -32)
    assert np.all(np.diff(f) > 0)


def test_collisions_above_one_256th():
    # Sec. 2.1: floats >= 1/256 necessarily collide: 2^24 and 2^24 + 1 both map to 2^-8,
    # and the 256 inputs 2^31 .. 2^31 + 255 all map to 1/2.
    f = map_u32_to_unifloat(np.array([1 << 24, (1 << 24) + 1], dtype=np.uint64))
    assert f[0] == f[1] == np.float32(2.0 ** -8)
    h = map_u32_to_unifloat(np.arange(1 << 31, (1 << 31) + 256, dtype=np.uint64))
    assert np.all(h == np.float32(0.5))
