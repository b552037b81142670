"""Seeded input generators (random draws and layouts only).

Seeds used by the standard workloads:
  0 direction numbers, 1 per-dimension scramble seeds, 2 per-dimension shifts,
  3 lattice generator vector, 4 per-pixel Genz parameters, 5 sample-count maps,
  6 Gaussian-lobe parameters, 7 target perturbation, 8 sampled parameter indices.
"""

import numpy as np

# Enough initial direction numbers for any primitive polynomial of degree <= 16.
MAX_DEGREE = 16

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed, n, stream=0):
    """n consecutive SplitMix64 outputs for generator state `seed` (uint64 array).

    `stream` offsets the counter so that independent draws from one seed do not
    overlap: output k is mix(seed + (stream * 2**32 + k + 1) * gamma).
    """
    k = np.arange(n, dtype=np.uint64) + np.uint64(1) + np.uint64(stream) * np.uint64(1 << 32)
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + k * _GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform01(seed, n, stream=0):
    """n doubles uniform on [0, 1), 53 random bits each."""
    return (splitmix64(seed, n, stream) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def u32_draws(seed, n, stream=0):
    """n uniform 32-bit integers (the high half of each SplitMix64 output)."""
    return (splitmix64(seed, n, stream) >> np.uint64(32)).astype(np.uint32)


def sobol_direction_init(s, seed=0):
    """Initial direction numbers m_1..m_MAX_DEGREE for s dimensions, uint32 [s][MAX_DEGREE].

    m_k is odd and below 2**k: m_k = 2 * (r mod 2**(k-1)) + 1 for a fresh 32-bit draw r.
    A dimension built from a degree-d polynomial uses the first d entries of its row.
    """
    r = u32_draws(seed, s * MAX_DEGREE).reshape(s, MAX_DEGREE).astype(np.uint64)
    k = np.arange(1, MAX_DEGREE + 1, dtype=np.uint64)
    mod = np.uint64(1) << (k - np.uint64(1))
    m = np.uint64(2) * (r % mod) + np.uint64(1)
    return m.astype(np.uint32)


def nus_seeds(s, seed=1):
    """One 32-bit scramble seed per dimension, uint32 [s]."""
    return u32_draws(seed, s)


def cp_shifts(s, seed=2):
    """One 32-bit rotation (shift) per dimension, uint32 [s]."""
    return u32_draws(seed, s)


def lattice_vector(s, bits, seed=3):
    """Generator vector with odd components uniform in [1, 2**bits), uint32 [s]."""
    r = u32_draws(seed, s).astype(np.uint64)
    g = np.uint64(2) * (r % (np.uint64(1) << np.uint64(bits - 1))) + np.uint64(1)
    return g.astype(np.uint32)


def genz_params(num_pixels, seed=4):
    """Per-pixel Genz parameters, float32 [P][16]: 8 centres U[0,1) then 8 widths U[2,20]."""
    u = uniform01(seed, num_pixels * 16).reshape(num_pixels, 16)
    out = np.empty((num_pixels, 16), dtype=np.float32)
    out[:, :8] = u[:, :8].astype(np.float32)
    out[:, 8:] = (2.0 + 18.0 * u[:, 8:]).astype(np.float32)
    # U[0,1) draws may round up to 1.0 in float32; keep centres strictly inside.
    out[:, :8] = np.minimum(out[:, :8], np.float32(np.nextafter(np.float32(1), np.float32(0))))
    return out


def value_noise(width, height, seed, cell=32):
    """Bilinear value noise in [0,1) on a `cell`-pixel lattice, float64 [height][width].

    Lattice values are uniform draws; pixel (x, y) is sampled at its centre.
    """
    gw = width // cell + 2
    gh = height // cell + 2
    lat = uniform01(seed, gw * gh).reshape(gh, gw)
    xs = (np.arange(width) + 0.5) / cell
    ys = (np.arange(height) + 0.5) / cell
    x0 = np.floor(xs).astype(np.int64)
    y0 = np.floor(ys).astype(np.int64)
    fx = xs - x0
    fy = ys - y0
    a = lat[np.ix_(y0, x0)]
    b = lat[np.ix_(y0, x0 + 1)]
    c = lat[np.ix_(y0 + 1, x0)]
    d = lat[np.ix_(y0 + 1, x0 + 1)]
    top = a + (b - a) * fx[None, :]
    bot = c + (d - c) * fx[None, :]
    v = top + (bot - top) * fy[:, None]
    return np.minimum(v, np.nextafter(1.0, 0.0))


def counts_pow2(width, height, seed=5, max_log2=8):
    """Adaptive per-pixel sample counts 2**k, k = min(max_log2, floor((max_log2+1) * v)).

    v is smooth value noise, so neighbouring pixels get similar counts; uint32 [H*W],
    row-major (pixel p = y * width + x).
    """
    v = value_noise(width, height, seed)
    k = np.minimum(max_log2, np.floor((max_log2 + 1) * v)).astype(np.uint32)
    return (np.uint32(1) << k).reshape(-1).astype(np.uint32)


def counts_progressive(width, height, seed=5, passes=16, spp_per_pass=64):
    """Counts spp_per_pass * c, c = 1 + min(passes-1, floor(passes * v)); uint32 [H*W]."""
    v = value_noise(width, height, seed)
    c = 1 + np.minimum(passes - 1, np.floor(passes * v)).astype(np.uint32)
    return (np.uint32(spp_per_pass) * c).reshape(-1).astype(np.uint32)


def counts_uniform(width, height, spp):
    """The same count for every pixel, uint32 [H*W]."""
    return np.full(width * height, spp, dtype=np.uint32)


def lobe_params(num_lobes, dim, seed=6):
    """Gaussian-lobe parameter vector theta, float32 [L*(2d+1)].

    Layout: centres [L][d] U[0,1), log-widths [L][d] = log(U[0.1,0.5] * sqrt(d/8)),
    weights [L] = U[0.5,1.5] / L.
    """
    L, d = num_lobes, dim
    u = uniform01(seed, L * (2 * d + 1))
    c = u[: L * d]
    sig = (0.1 + 0.4 * u[L * d: 2 * L * d]) * np.sqrt(d / 8.0)
    w = (0.5 + u[2 * L * d:]) / L
    theta = np.concatenate([c, np.log(sig), w]).astype(np.float32)
    theta[: L * d] = np.minimum(theta[: L * d], np.float32(np.nextafter(np.float32(1), np.float32(0))))
    return theta


def perturb(theta, seed=7, rel=0.05):
    """theta * (1 + U[-rel, rel]) elementwise, float32."""
    u = uniform01(seed, theta.size)
    return (theta.astype(np.float64) * (1.0 + rel * (2.0 * u - 1.0))).astype(np.float32)


def pick(n_total, k, seed=8):
    """k distinct indices in [0, n_total), sorted (partial Fisher-Yates on SplitMix64 draws)."""
    k = min(k, n_total)
    r = splitmix64(seed, k)
    chosen = {}
    out = []
    for t in range(k):
        j = t + int(r[t] % np.uint64(n_total - t))
        vt = chosen.get(t, t)
        vj = chosen.get(j, j)
        chosen[j] = vt
        chosen[t] = vj
        out.append(vj)
    return np.array(sorted(out), dtype=np.int64)
