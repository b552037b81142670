"""GPU parity of the Halton sequence (Sec. 2.2): every u32 and float32 value bit-exact against
the oracle, at sizes the oracle finishes quickly, on sampled entries of the 2^24 x 32 launch,
and by the stratification property at sizes beyond the oracle."""

import numpy as np
import pytest

from oracle import halton, unifloat
from synth import u32_draws

pytestmark = pytest.mark.gpu

MODES = {"identity": 0, "faure": 1, "linear": 2}


def _factors(s):
    return (u32_draws(11, s) | 1).astype(np.uint32)


def _run(q, s, first, n, mode, ld=None):
    import torch

    f = _factors(s)
    df = q.from_u32(f) if mode == "linear" else None
    u, x = q.qmc_generate_halton(s, first, n, MODES[mode], df, ld=ld)
    torch.cuda.synchronize()
    gu = q.to_u32(u)[:, :n]
    gx = x.cpu().numpy()[:, :n].view(np.uint32)
    eu = halton.halton_points(s, first, n, mode, f if mode == "linear" else None)
    ex = unifloat.map_u32_to_unifloat(eu).view(np.uint32)
    return gu, gx, eu, ex


CASES = [
    # s, first, n, mode, ld
    (8, 0, 3000, "identity", None),           # several wave runs, ragged tail
    (16, 4 * 1001, 2001, "faure", None),      # aligned start off a chunk boundary
    (5, 7, 999, "linear", None),              # unaligned start: general kernel
    (64, 0, 600, "faure", None),              # all 64 bases (2 .. 311)
    (3, 3486784401 - 100, 400, "identity", None),   # across the base-3 index reduction
    (2, (1 << 32) - 2000, 2000, "linear", None),    # top of the 32-bit index range
    (6, 256, 1000, "faure", 1030),            # leading dimension > n
]


@pytest.mark.parametrize("s,first,n,mode,ld", CASES)
def test_halton_bit_exact(qmc, s, first, n, mode, ld):
    gu, gx, eu, ex = _run(qmc, s, first, n, mode, ld)
    assert np.array_equal(gu, eu), (s, first, n, mode)
    assert np.array_equal(gx, ex), (s, first, n, mode)


@pytest.mark.parametrize("mode", ["identity", "faure", "linear"])
def test_halton_full_size_sampled(qmc, mode):
    """The 2^24 x 32 launch (the generation benchmark's size): 3000 sampled entries."""
    import torch

    s, n = 32, 1 << 24
    f = _factors(s)
    u, _ = qmc.qmc_generate_halton(s, 0, n, MODES[mode], qmc.from_u32(f) if mode == "linear" else None,
                                   want_f32=False)
    torch.cuda.synchronize()
    rng = np.random.default_rng(3)
    js = rng.integers(0, s, 3000)
    iis = rng.integers(0, n, 3000)
    got = qmc.to_u32(u[torch.from_numpy(js).cuda(), torch.from_numpy(iis).cuda()].reshape(1, -1))[0]
    bases = halton.primes(s)
    for k in range(3000):
        j, i = int(js[k]), int(iis[k])
        sig = halton.digit_permutation(bases[j], mode, int(f[j]))
        assert int(got[k]) == halton.radical_inverse_u32(i, bases[j], sig), (j, i)


def test_halton_first_b_power_points_stratify_at_scale(qmc):
    """phi_b of i < b^m is one point per cell k / b^m: checked on 3^12, 5^8 and 7^7 points."""
    import torch

    for j, b, m in ((1, 3, 12), (2, 5, 8), (3, 7, 7)):
        n = b ** m
        u, _ = qmc.qmc_generate_halton(4, 0, n, 1, None, want_f32=False)
        torch.cuda.synchronize()
        got = np.sort(qmc.to_u32(u)[j, :n].astype(np.uint64))
        want = (np.arange(n, dtype=np.uint64) << np.uint64(32)) // np.uint64(n)
        assert np.array_equal(got, want), (b, m)


def _just_below_a_grid_point(b, sig):
    """The index x < b^M whose value lies closest below a multiple of 2^-32: its mirrored digit
    value R has 2^32 R = -1 mod b^M.  There the table-driven kernel's 64-bit fixed-point sum
    cannot decide the last bit for some bases and the exact digit loop takes over."""
    bm = halton.max_power(b)
    digits = 0
    while b ** (digits + 1) <= bm:
        digits += 1
    r = (-pow(1 << 32, -1, bm)) % bm
    inv = {v: a for a, v in enumerate(sig)}
    x = 0
    for p in range(digits):          # digit p of R (lowest first) is sigma(a_(digits-1-p))
        r, d = divmod(r, b)
        x += inv[d] * b ** (digits - 1 - p)
    return x


@pytest.mark.parametrize("mode", ["identity", "faure"])
def test_halton_near_grid_points_every_base(qmc, mode):
    import torch

    bases = halton.primes(64)
    for j in range(1, 64):
        b = bases[j]
        sig = halton.digit_permutation(b, mode)
        x = _just_below_a_grid_point(b, sig)
        first = max(0, (x & ~3) - 128)
        n = 256
        u, _ = qmc.qmc_generate_halton(j + 1, first, n, MODES[mode], None, want_f32=False)
        torch.cuda.synchronize()
        got = qmc.to_u32(u)[j, :n]
        want = [halton.radical_inverse_u32(first + t, b, sig) for t in range(n)]
        assert [int(v) for v in got] == want, (b, x)


def test_halton_argument_errors(qmc):
    with pytest.raises(qmc.QMCError) as e:
        qmc.qmc_generate_halton(4, 0, 100, 3)
    assert e.value.status == 1
    with pytest.raises(qmc.QMCError) as e:
        qmc.qmc_generate_halton(4, 0, 100, 2, None)
    assert e.value.status == 1
    with pytest.raises(qmc.QMCError) as e:
        qmc.qmc_generate_halton(65, 0, 10, 0)
    assert e.value.status == 2
    with pytest.raises(qmc.QMCError) as e:
        qmc.qmc_generate_halton(4, (1 << 32) - 10, 11, 0)
    assert e.value.status == 2
