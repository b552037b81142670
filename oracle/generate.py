"""Materialised point sets: the batched form of the per-component functions of Alg. 3
(Sobol') and Alg. 4 (rank-1 lattice), randomised in integers (Sec. 2.1, 2.3) and then
converted with map_u32_to_unifloat (Alg. 1).

Layout of a result: dimension-major, out[j][i - first].
Sobol':  v = C_j a(i);  NUS_{nus_seeds[j]}(v) if seeds are given;  shift if shifts are given.
Lattice: v = (phi_2(i) g_j) mod 1 (backward: phi_2(2^32 - 1 - i));  shift if given.
The shift is (v + delta_j) mod 2^32 unless SHIFT_XOR is set, then v ^ delta_j.
"""

import numpy as np

from . import digital, lattice, scramble, unifloat

SHIFT_XOR = 1
LATTICE_BACKWARD = 2


def _shift(v, delta, flags):
    return scramble.shift_xor(v, delta) if flags & SHIFT_XOR else scramble.shift_add(v, delta)


def sobol_at(mats, idx, nus_seeds=None, shifts=None, flags=0, dims=None):
    """uint32 [len(dims)][len(idx)] for arbitrary indices idx."""
    idx = np.asarray(idx, dtype=np.uint64)
    dims = range(mats.shape[0]) if dims is None else dims
    rows = []
    for j in dims:
        v = digital.digital_point(mats[j], idx)
        if nus_seeds is not None:
            v = scramble.nested_uniform_scramble(v, int(nus_seeds[j]))
        if shifts is not None:
            v = _shift(v, int(shifts[j]), flags)
        rows.append(v.astype(np.uint32))
    return np.stack(rows) if rows else np.zeros((0, idx.size), np.uint32)


def lattice_at(g, idx, shifts=None, flags=0, dims=None):
    """uint32 [len(dims)][len(idx)] for arbitrary indices idx."""
    idx = np.asarray(idx, dtype=np.uint64)
    dims = range(len(g)) if dims is None else dims
    rows = []
    for j in dims:
        v = lattice.lattice_point(int(g[j]), idx, backward=bool(flags & LATTICE_BACKWARD))
        if shifts is not None:
            v = _shift(v, int(shifts[j]), flags)
        rows.append(v.astype(np.uint32))
    return np.stack(rows) if rows else np.zeros((0, idx.size), np.uint32)


def generate_sobol(mats, first, n, nus_seeds=None, shifts=None, flags=0):
    """(u32 [s][n], f32 [s][n]) for i in [first, first+n)."""
    idx = np.arange(n, dtype=np.uint64) + np.uint64(first)
    u = sobol_at(mats, idx, nus_seeds, shifts, flags)
    return u, unifloat.map_u32_to_unifloat(u)


def generate_lattice(g, first, n, shifts=None, flags=0):
    """(u32 [s][n], f32 [s][n]) for i in [first, first+n)."""
    idx = np.arange(n, dtype=np.uint64) + np.uint64(first)
    u = lattice_at(g, idx, shifts, flags)
    return u, unifloat.map_u32_to_unifloat(u)
