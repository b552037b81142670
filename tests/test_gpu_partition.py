"""GPU parity of 64-bit indices and partitioned enumeration (Sec. 2.5.1, Alg. 3's 64-bit index,
Eq. R1LS over 64 digits): every u32 and float32 value bit-exact against the oracle at sizes it
finishes quickly, sampled entries of the 2^24 x 32 launches, and the piece split beyond 2^31
points."""

import numpy as np
import pytest

from oracle import partition, scramble, unifloat
from synth import cp_shifts, lattice_vector, nus_seeds, sobol_direction_init

pytestmark = pytest.mark.gpu

XOR = partition.SHIFT_XOR
BACK = partition.LATTICE_BACKWARD
P64 = 1 << 64


def _mats(s, columns):
    return partition.sobol_matrices_wide(s, sobol_direction_init(s, 0), columns)


def _host(q, u, f, n):
    import torch

    torch.cuda.synchronize()
    gu = q.to_u32(u)[:, :n] if u is not None else None
    gf = f.cpu().numpy()[:, :n].view(np.uint32) if f is not None else None
    return gu, gf


SOBOL_CASES = [
    # s, columns, log2_parts, part, first, n, nus, shift, flags, ld
    (4, 64, 0, 0, 1 << 40, 3000, True, True, 0, None),                  # whole sequence past 2^32
    (8, 52, 5, 19, (1 << 40) + 4 * 1001, 3001, True, False, 0, None),   # start off a 256 boundary
    (3, 64, 32, 0xDEADBEEF, (1 << 32) - 2400, 2000, False, True, XOR, None),  # m crosses 2^32
    (2, 36, 32, 5, 0, 16, False, False, 0, None),                       # the whole part (2^4 points)
    (5, 64, 8, 200, (1 << 56) - 1200, 1200, True, True, 0, None),       # top of a part's range
    (3, 64, 0, 0, P64 - 1000, 1000, True, True, 0, None),               # top of the 64-bit range
    (6, 64, 3, 6, 7, 999, True, False, 0, None),                        # unaligned start: general kernel
    (4, 48, 2, 3, 1 << 33, 2000, True, True, XOR, 2003),                # odd ld: general kernel
    (9, 64, 1, 1, 256, 3000, True, True, 0, 3004),                      # ld > n, aligned
]


@pytest.mark.parametrize("case", SOBOL_CASES, ids=[str(c[:5]) for c in SOBOL_CASES])
def test_sobol64_bit_exact(qmc, case):
    s, columns, lq, part, first, n, nus, shift, flags, ld = case
    mats = _mats(s, columns)
    seeds = nus_seeds(s, 1) if nus else None
    shifts = cp_shifts(s, 2) if shift else None
    u, f = qmc.qmc_generate_sobol64(qmc.from_u32(mats), first, n, lq, part,
                                    qmc.from_u32(seeds) if nus else None, qmc.from_u32(shifts) if shift else None,
                                    flags, ld=ld)
    gu, gf = _host(qmc, u, f, n)
    eu, ef = partition.generate_sobol64(mats, lq, part, first, n, seeds, shifts, flags)
    assert np.array_equal(gu, eu), case
    assert np.array_equal(gf, ef.view(np.uint32)), case


LATTICE_CASES = [
    # s, log2_parts, part, first, n, shift, flags
    (4, 0, 0, 1 << 40, 3000, False, 0),
    (6, 7, 100, (1 << 50) + 8, 3001, True, BACK),
    (3, 32, 77, (1 << 32) - 2400, 2000, True, XOR),
    (5, 3, 2, 13, 999, False, 0),                  # unaligned start: general kernel
    (2, 0, 0, P64 - 1000, 1000, False, BACK),       # top of the 64-bit range
    (3, 12, 4000, (1 << 52) - 1000, 1000, True, 0),  # top of a part's range
]


@pytest.mark.parametrize("case", LATTICE_CASES, ids=[str(c[:4]) for c in LATTICE_CASES])
def test_lattice64_bit_exact(qmc, case):
    s, lq, part, first, n, shift, flags = case
    g = lattice_vector(s, 30, 5)
    shifts = cp_shifts(s, 2) if shift else None
    u, f = qmc.qmc_generate_lattice64(qmc.from_u32(g), first, n, lq, part,
                                      qmc.from_u32(shifts) if shift else None, flags)
    gu, gf = _host(qmc, u, f, n)
    eu, ef = partition.generate_lattice64(g, lq, part, first, n, shifts, flags)
    assert np.array_equal(gu, eu), case
    assert np.array_equal(gf, ef.view(np.uint32)), case


def test_one_part_below_2p32_equals_the_32_bit_calls(qmc):
    """log2_parts = 0 and indices below 2^32: the same points as qmc_generate_sobol /
    qmc_generate_lattice (forward)."""
    import torch

    s, first, n = 16, 4 * 5000, 20000
    wide = _mats(s, 64)
    seeds, shifts = qmc.from_u32(nus_seeds(s, 1)), qmc.from_u32(cp_shifts(s, 2))
    a, _ = qmc.qmc_generate_sobol64(qmc.from_u32(wide), first, n, 0, 0, seeds, shifts, want_f32=False)
    b, _ = qmc.qmc_generate_sobol(qmc.from_u32(wide[:, :32].copy()), first, n, seeds, shifts, want_f32=False)
    g = qmc.from_u32(lattice_vector(s, 20, 3))
    c, _ = qmc.qmc_generate_lattice64(g, first, n, 0, 0, shifts, want_f32=False)
    d, _ = qmc.qmc_generate_lattice(g, first, n, shifts, want_f32=False)
    torch.cuda.synchronize()
    assert torch.equal(a, b) and torch.equal(c, d)


def test_parts_interleave_into_the_sequence(qmc):
    """The 2^q parts, each enumerated from m = 0, hold every index exactly once:
    part p's m-th point is the sequence's point m 2^q + rev_q(p)."""
    import torch

    s, q, per = 5, 4, 512
    mats = qmc.from_u32(_mats(s, 64))
    whole, _ = qmc.qmc_generate_sobol64(mats, 0, per << q, want_f32=False)
    for p in range(1 << q):
        part, _ = qmc.qmc_generate_sobol64(mats, 0, per, q, p, want_f32=False)
        r = partition.rev_bits(p, q)
        torch.cuda.synchronize()
        assert torch.equal(part, whole[:, r::1 << q]), p


def _sampled(rng, s, n, k=3000):
    return rng.integers(0, s, k), rng.integers(0, n, k)


def test_sobol64_full_size_sampled(qmc):
    """2^24 points x 32 dims of part 77 of 2^8, starting at m = 2^44: 3000 sampled entries."""
    import torch

    s, n, lq, part, first = 32, 1 << 24, 8, 77, 1 << 44
    mats = _mats(s, 64)
    seeds, shifts = nus_seeds(s, 1), cp_shifts(s, 2)
    u, f = qmc.qmc_generate_sobol64(qmc.from_u32(mats), first, n, lq, part, qmc.from_u32(seeds),
                                    qmc.from_u32(shifts))
    js, ts = _sampled(np.random.default_rng(5), s, n)
    dj, dt = torch.from_numpy(js).cuda(), torch.from_numpy(ts).cuda()
    gu = qmc.to_u32(u[dj, dt].reshape(1, -1))[0]
    gf = f[dj, dt].cpu().numpy().view(np.uint32)
    for k in range(len(js)):
        j, t = int(js[k]), int(ts[k])
        v = partition.digital_point64(mats[j], partition.part_index(lq, part, first + t))
        v = int(scramble.nested_uniform_scramble(np.uint64(v), int(seeds[j])))
        v = (v + int(shifts[j])) & 0xFFFFFFFF
        assert int(gu[k]) == v, (j, t)
        assert int(gf[k]) == int(unifloat.map_u32_to_unifloat_bits(np.uint32(v))), (j, t)


def test_lattice64_full_size_sampled(qmc):
    import torch

    s, n, lq, part, first = 32, 1 << 24, 10, 999, 1 << 50
    g = lattice_vector(s, 30, 5)
    u, _ = qmc.qmc_generate_lattice64(qmc.from_u32(g), first, n, lq, part, want_f32=False)
    js, ts = _sampled(np.random.default_rng(6), s, n)
    gu = qmc.to_u32(u[torch.from_numpy(js).cuda(), torch.from_numpy(ts).cuda()].reshape(1, -1))[0]
    for k in range(len(js)):
        j, t = int(js[k]), int(ts[k])
        assert int(gu[k]) == partition.lattice_point64(int(g[j]), partition.part_index(lq, part, first + t)), (j, t)


def test_more_than_2p31_points_in_one_call(qmc):
    """n = 2^31 + 1000 (launched in pieces of 2^31): entries around the piece boundary and the end."""
    import torch

    n, first, lq, part = (1 << 31) + 1000, 1 << 36, 2, 1
    mats = _mats(1, 64)
    u, _ = qmc.qmc_generate_sobol64(qmc.from_u32(mats), first, n, lq, part, want_f32=False)
    ts = np.array([0, 1, 2, (1 << 31) - 3, (1 << 31) - 1, 1 << 31, (1 << 31) + 1, n - 2, n - 1], np.int64)
    gu = qmc.to_u32(u[0, torch.from_numpy(ts).cuda()].reshape(1, -1))[0]
    del u
    torch.cuda.empty_cache()
    for k, t in enumerate(ts):
        assert int(gu[k]) == partition.digital_point64(mats[0], partition.part_index(lq, part, first + int(t))), t


def test_argument_errors(qmc):
    import torch

    m64 = qmc.from_u32(_mats(4, 64))
    m40 = qmc.from_u32(_mats(4, 40))
    g = qmc.from_u32(lattice_vector(4, 30, 5))

    def status(fn, *a, **k):
        with pytest.raises(qmc.QMCError) as e:
            fn(*a, **k)
        return e.value.status

    assert status(qmc.qmc_generate_sobol64, m64, 0, 16, 33, 0) == 2           # more than 2^32 parts
    assert status(qmc.qmc_generate_sobol64, m40, 0, 16, 3, 8) == 2            # part >= 2^q
    assert status(qmc.qmc_generate_sobol64, m40, 1 << 37, 1, 3, 0) == 2       # m beyond 2^(40 - 3)
    assert status(qmc.qmc_generate_sobol64, m40, (1 << 37) - 4, 5, 3, 0) == 2
    assert status(qmc.qmc_generate_sobol64, m64, 0, 16, 0, 0, flags=128) == 1  # point-major not here
    assert status(qmc.qmc_generate_lattice64, g, P64 - 4, 5, 0, 0) == 2
    assert status(qmc.qmc_generate_lattice64, g, 1 << 40, 16, 30, 0) == 2     # m beyond 2^34
    assert status(qmc.qmc_generate_lattice64, g, 0, 16, 0, 0, flags=128) == 1
    # the last admissible indices are accepted
    u, _ = qmc.qmc_generate_sobol64(m40, (1 << 37) - 4, 4, 3, 7, want_f32=False)
    v, _ = qmc.qmc_generate_lattice64(g, (1 << 34) - 4, 4, 30, 5, want_f32=False)
    torch.cuda.synchronize()
    assert u.shape == (4, 4) and v.shape == (4, 4)
