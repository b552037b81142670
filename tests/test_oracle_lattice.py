"""Pins for the oracle's rank-1 lattice sequences (Sec. 2.4, Eq. R1LS, Alg. 4)."""

import numpy as np

from oracle import lattice
from synth import lattice_vector


def _rev(v, bits):
    return int(format(int(v), "0%db" % bits)[::-1], 2)


def test_closed_form_k_g_over_n():
    # First n = 2^20 points: phi_2(i) * 2^20 = rev20(i) =: k, x = (k g mod n) / n.
    g = lattice_vector(32, 20, 3)
    i = np.arange(0, 1 << 20, 997, dtype=np.uint64)
    pts = lattice.lattice_points(g, 0, 1 << 20)[:, i.astype(np.int64)].astype(np.uint64)
    for col, iv in enumerate(i[:300]):
        k = _rev(iv, 20)
        for j in range(0, 32, 7):
            assert int(pts[j, col]) == ((k * int(g[j])) % (1 << 20)) << 12


def test_latin_hypercube_for_odd_generators():
    # Odd g_j: each dimension of the first 2^m points is a permutation of {k / 2^m}.
    g = lattice_vector(8, 20, 3)
    for m in (4, 10, 16):
        pts = lattice.lattice_points(g, 0, 1 << m).astype(np.uint64)
        for j in range(8):
            assert np.unique(pts[j] >> np.uint64(32 - m)).size == 1 << m
            assert np.all(pts[j] & np.uint64((1 << (32 - m)) - 1) == 0)


def test_point_set_is_a_rank1_lattice_rule():
    g = lattice_vector(4, 20, 3)
    m = 12
    n = 1 << m
    pts = lattice.lattice_points(g, 0, n).astype(np.uint64)
    got = sorted(tuple(int(v) for v in pts[:, c]) for c in range(n))
    want = sorted(tuple(((k * int(gj)) % n) << (32 - m) for gj in g) for k in range(n))
    assert got == want


def test_backward_enumeration_puts_origin_last():
    g = lattice_vector(4, 20, 3)
    last = lattice.lattice_points(g, 0xFFFFFFFF, 1, backward=True)
    assert np.all(last == 0)
    first = lattice.lattice_points(g, 0, 1, backward=True).astype(np.uint64)
    assert np.array_equal(first[:, 0], (np.uint64(0xFFFFFFFF) * g.astype(np.uint64)) & np.uint64(0xFFFFFFFF))


def test_shifted_lattice_decomposition():
    # Sec. 2.4.1: phi_2(i + k 2^m) = phi_2(i) + phi_2(k) 2^-m for i < 2^m (the exponent is
    # -m; the printed -m-1 is off by one), so block k is block 0 shifted by that amount times g.
    from oracle.digital import radical_inverse_base2 as rb
    m = 10
    i = np.arange(1 << m, dtype=np.uint64)
    for k in (1, 2, 3, 77, 1000):
        lhs = rb(i + np.uint64(k << m))
        rhs = rb(i) + (rb(np.array([k], dtype=np.uint64)) >> np.uint64(m))
        assert np.array_equal(lhs, rhs)
