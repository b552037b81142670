"""Per-pixel QMC integro-approximation (Sec. 2.5: one randomised copy of the sequence per
processing element, here per pixel; no communication until the final reduction).

Pixel p = y * width + x (row-major) integrates with samples i in [0, N_p), N_p = counts[p].
Sample i of pixel p, dimension j (all integer until the last step, Sec. 2.1):
  Sobol':  v = C_j a(i);  v = NUS_{seed_pj}(v) if scrambling;  v = shift(v, delta_pj) if shifting
  lattice: v = ((phi_2(i) + s_p) g_j) mod 1 (or backward);   v = shift(v, delta_pj) if shifting
  x = map_u32_to_unifloat(v)
with seed_pj = H(H(seed + 2j) ^ p) and delta_pj = H(H(seed + 2j + 1) ^ p).  The lattice
options of Sec. 3 (see pixel_lattice): g_j may be replaced by the per-pixel random generator
g_pj (Alg. 4), optionally with four superimposed instances, and s_p is the pixel's Hilbert
shift floor(2^32 phi_3(h(x, y))) (Eq. PixelShiftedR1LS), else 0.
  With PIXEL_TABLE_SHIFT the rotation delta_pj is entry j mod 2 of the pixel's cell in a
  128 x 128 table of two-dimensional shifts (Sec. 2.6.1, see xor_table).
  XOR table (Sec. 2.6.1, see xor_table): v = P_j[(i XOR r_c) mod N] XOR s_cj for the pixel's
  cell c in the 128 x 128 tables.

A call covers the window of sample indices [begin, min(end, N_p)); the window sum is
added to `sums` and the mean is sums / N_p.  The estimator I_p = (1/N_p) sum_i f_p(x_pi)
is evaluated in FP64 at the float32 points (promoted exactly), each pixel's sum taken
with math.fsum (correctly rounded, hence independent of order).
"""

import math

import numpy as np

from . import digital, lattice, pixel_lattice, scramble, unifloat, xor_table
from .integrands import genz, lobes, lobes_weighted_gradient, lobes_weighted_gradient_abs

# Flag bits shared with the library's public header (values fixed by that interface).
SHIFT_XOR = 1
LATTICE_BACKWARD = 2
PIXEL_NUS = 4
PIXEL_SHIFT = 8
PIXEL_RANDOM_GENERATOR = 16
PIXEL_HILBERT_SHIFT = 32
LATTICE_INSTANCES4 = 64
PIXEL_TABLE_SHIFT = 256


def window_pairs(counts, pixels, begin, end):
    """(pixel index array, sample index array, per-pixel segment starts) of a window."""
    counts = np.asarray(counts, dtype=np.int64)
    ps, idx, starts = [], [], [0]
    for p in pixels:
        lo = begin
        hi = min(end, int(counts[p]))
        n = max(0, hi - lo)
        ps.append(np.full(n, p, dtype=np.int64))
        idx.append(np.arange(lo, lo + n, dtype=np.int64))
        starts.append(starts[-1] + n)
    if ps:
        return np.concatenate(ps), np.concatenate(idx), np.array(starts)
    return np.zeros(0, np.int64), np.zeros(0, np.int64), np.array([0])


def pixel_samples_u32(sampler, p, i):
    """Integer sample components, uint32 [s][n], for pixel/index arrays p, i."""
    kind = sampler["kind"]
    if kind == "xor_table":
        # Sec. 2.6.1: stored points reindexed and scrambled per pixel from 128 x 128 tables
        return xor_table.xor_table_samples_u32(sampler["table"], sampler["scramble"], sampler["reorder"],
                                               sampler["width"], p, i)
    s = sampler["s"]
    flags = sampler.get("flags", 0)
    seed = sampler.get("seed", 0)
    table = sampler["table"]
    p = np.asarray(p, dtype=np.uint64)
    i = np.asarray(i, dtype=np.uint64)
    out = np.zeros((s, p.size), dtype=np.uint32)
    for j in range(s):
        if kind == "sobol":
            v = digital.digital_point(table[j], i)
            if flags & PIXEL_NUS:
                v = scramble.nested_uniform_scramble(v, scramble.pixel_nus_seed(seed, p, j))
        elif kind == "lattice":
            v = _pixel_lattice_component(sampler, p, i, j)
        else:
            raise ValueError(kind)
        if flags & PIXEL_SHIFT:
            if flags & PIXEL_TABLE_SHIFT:
                d = xor_table.table_shift(sampler["shift_table"], sampler["width"], p, j)
            else:
                d = scramble.pixel_shift(seed, p, j)
            v = scramble.shift_xor(v, d) if flags & SHIFT_XOR else scramble.shift_add(v, d)
        out[j] = v.astype(np.uint32)
    return out


def _pixel_lattice_component(sampler, p, i, j):
    """Component j of the lattice samples (Sec. 2.4; Alg. 4 and Eq. PixelShiftedR1LS options)."""
    flags = sampler.get("flags", 0)
    back = bool(flags & LATTICE_BACKWARD)
    if not flags & (PIXEL_RANDOM_GENERATOR | PIXEL_HILBERT_SHIFT | LATTICE_INSTANCES4):
        return lattice.lattice_point(sampler["table"][j], i, backward=back)
    inst = i & np.uint64(3) if flags & LATTICE_INSTANCES4 else np.zeros_like(i)
    idx = i >> np.uint64(2) if flags & LATTICE_INSTANCES4 else i
    v = np.zeros(p.size, dtype=np.uint64)
    keys = np.stack([p, inst]) if p.size else np.zeros((2, 0), np.uint64)
    for pp, c in {(int(a), int(b)) for a, b in keys.T}:
        sel = (p == np.uint64(pp)) & (inst == np.uint64(c))
        if flags & PIXEL_RANDOM_GENERATOR:
            g = pixel_lattice.pixel_generator(sampler.get("seed", 0), pp, j, c)
        else:
            g = int(sampler["table"][j])
        sh = (pixel_lattice.pixel_hilbert_shift(pp, sampler["width"], sampler["height"])
              if flags & PIXEL_HILBERT_SHIFT else 0)
        v[sel] = pixel_lattice.pixel_lattice_points(g, idx[sel], sh, back)
    return v


def pixel_samples_f32(sampler, p, i):
    """Float sample components in [0,1), float32 [s][n]."""
    return unifloat.map_u32_to_unifloat(pixel_samples_u32(sampler, p, i))


def pixel_offsets(pixel_seed, p, dim):
    """Per-pixel integrand offsets delta_pj in [-1/4, 1/4), float32 [d][n].

    delta = fl32(fl32(0.5 * map_u32_to_unifloat(H(H(pixel_seed + j) ^ p))) - 0.25),
    each operation rounded to nearest in binary32.
    """
    p = np.asarray(p, dtype=np.uint64)
    out = np.zeros((dim, p.size), dtype=np.float32)
    for j in range(dim):
        u = unifloat.map_u32_to_unifloat(scramble.pixel_offset_u32(pixel_seed, p, j))
        out[j] = (np.float32(0.5) * u).astype(np.float32) - np.float32(0.25)
    return out


def integrand_values(integrand, x32, p, theta=None):
    """(f, envelope) in FP64 at float32 points x32 [s][n] belonging to pixels p."""
    kind = integrand["kind"]
    if kind == "genz":
        pp = np.asarray(integrand["pixel_params"], dtype=np.float32)[np.asarray(p, dtype=np.int64)]
        return genz(x32[:8].astype(np.float64), pp.astype(np.float64))
    if kind == "lobes":
        L, d = integrand["num_lobes"], integrand["d"]
        th = integrand["params"] if theta is None else theta
        y = x32[:d].astype(np.float64) + pixel_offsets(integrand["pixel_seed"], p, d).astype(np.float64)
        f = lobes(y, np.asarray(th, dtype=np.float64), L, d)
        return f, np.abs(f)
    raise ValueError(kind)


def segment_fsum(values, starts):
    """Correctly rounded sum of each segment values[starts[k]:starts[k+1]]."""
    return np.array([math.fsum(values[starts[k]:starts[k + 1]]) for k in range(len(starts) - 1)])


def integrate_pixels(sampler, integrand, counts, pixels, begin=0, end=2**32, theta=None):
    """Window sums, means and envelope means (FP64) for the listed pixels.

    Returns dict(sum, mean, env) with one entry per listed pixel; mean = sum / N_p
    (the full-window estimate when [begin, end) covers [0, N_p)), env = (1/N_p) * the
    window sum of the envelope bound |f| <= env.
    """
    pixels = np.asarray(pixels, dtype=np.int64)
    p, i, starts = window_pairs(counts, pixels, begin, end)
    x32 = pixel_samples_f32(sampler, p, i)
    f, env = integrand_values(integrand, x32, p, theta)
    sums = segment_fsum(f, starts)
    envs = segment_fsum(env, starts)
    n = np.asarray(counts, dtype=np.float64)[pixels]
    with np.errstate(invalid="ignore", divide="ignore"):
        mean = np.where(n > 0, sums / np.maximum(n, 1), 0.0)
        envm = np.where(n > 0, envs / np.maximum(n, 1), 0.0)
    return {"sum": sums, "mean": mean, "env": envm}


def l2_loss(means, target):
    """L = (1/P) sum_p (I_p - T_p)^2 over the listed pixels."""
    d = np.asarray(means, dtype=np.float64) - np.asarray(target, dtype=np.float64)
    return math.fsum(d * d) / d.size


def lobes_gradient(sampler, integrand, counts, pixels, grad_means, begin=0, end=2**32, theta=None, sizes=False):
    """dL/dtheta = sum_p gI_p (1/N_p) sum_{i in window} df(x_pi)/dtheta, FP64 [L*(2d+1)].

    With sizes=True, the sum of the absolute values of those terms instead: the scale of what an
    FP32 evaluation adds up, which bounds its rounding error (a test tolerance, not the method)."""
    pixels = np.asarray(pixels, dtype=np.int64)
    L, d = integrand["num_lobes"], integrand["d"]
    th = np.asarray(integrand["params"] if theta is None else theta, dtype=np.float64)
    p, i, starts = window_pairs(counts, pixels, begin, end)
    x32 = pixel_samples_f32(sampler, p, i)
    y = x32[:d].astype(np.float64) + pixel_offsets(integrand["pixel_seed"], p, d).astype(np.float64)
    n = np.asarray(counts, dtype=np.float64)
    gm = np.asarray(grad_means, dtype=np.float64)
    pos = {int(q): k for k, q in enumerate(pixels)}
    scale = np.array([gm[pos[int(q)]] / n[int(q)] for q in p]) if p.size else np.zeros(0)
    if sizes:
        return lobes_weighted_gradient_abs(y, scale, th, L, d)
    return lobes_weighted_gradient(y, scale, th, L, d)


def l2_gradient_term_sizes(sampler, integrand, counts, pixels, target):
    """Per parameter, sum_p (2/P)(|I_p - T_p| + |I_p|)(1/N_p) sum_i |df(x_pi)/dtheta|: the size of
    what an FP32 evaluation of the L2 gradient adds up (its dL/dI_p carries an error relative
    to |I_p|), so eps-scaled it bounds the rounding error of components that cancel.  A test
    tolerance, not part of the method."""
    pixels = np.asarray(pixels, dtype=np.int64)
    L, d = integrand["num_lobes"], integrand["d"]
    means = integrate_pixels(sampler, integrand, counts, pixels)["mean"]
    wgt = 2.0 * (np.abs(means - np.asarray(target, dtype=np.float64)) + np.abs(means)) / len(pixels)
    p, i, starts = window_pairs(counts, pixels, 0, 2**32)
    x32 = pixel_samples_f32(sampler, p, i)
    y = x32[:d].astype(np.float64) + pixel_offsets(integrand["pixel_seed"], p, d).astype(np.float64)
    n = np.asarray(counts, dtype=np.float64)
    pos = {int(q): k for k, q in enumerate(pixels)}
    scale = np.array([wgt[pos[int(q)]] / n[int(q)] for q in p]) if p.size else np.zeros(0)
    return lobes_weighted_gradient_abs(y, scale, np.asarray(integrand["params"], np.float64), L, d)


def loss_and_gradient(sampler, integrand, counts, pixels, target, theta=None):
    """(L, dL/dtheta, means) for the L2 loss against `target` over the listed pixels."""
    r = integrate_pixels(sampler, integrand, counts, pixels, theta=theta)
    means = r["mean"]
    loss = l2_loss(means, target)
    grad_means = 2.0 * (means - np.asarray(target, dtype=np.float64)) / len(pixels)
    g = lobes_gradient(sampler, integrand, counts, pixels, grad_means, theta=theta)
    return loss, g, means


def finite_difference(sampler, integrand, counts, pixels, target, indices, rel_step=1e-4):
    """Central differences of the FP64 loss for the listed parameter indices.

    h_k = rel_step * max(1, |theta_k|); the points do not depend on theta, so they are
    computed once.
    """
    pixels = np.asarray(pixels, dtype=np.int64)
    L, d = integrand["num_lobes"], integrand["d"]
    th0 = np.asarray(integrand["params"], dtype=np.float64)
    p, i, starts = window_pairs(counts, pixels, 0, 2**32)
    x32 = pixel_samples_f32(sampler, p, i)
    y = x32[:d].astype(np.float64) + pixel_offsets(integrand["pixel_seed"], p, d).astype(np.float64)
    n = np.asarray(counts, dtype=np.float64)[pixels]
    tgt = np.asarray(target, dtype=np.float64)

    def loss_at(th):
        f = lobes(y, th, L, d)
        means = segment_fsum(f, starts) / n
        return l2_loss(means, tgt)

    out = []
    for k in indices:
        h = rel_step * max(1.0, abs(th0[k]))
        tp = th0.copy()
        tm = th0.copy()
        tp[k] += h
        tm[k] -= h
        out.append((loss_at(tp) - loss_at(tm)) / (2.0 * h))
    return np.array(out)
