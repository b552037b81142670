"""GPU parity of point generation against the CPU oracle (bit-exact, Sec. 2.1-2.4)."""

import os

import numpy as np
import pytest

from _exhaustive import compare_slice
from oracle import digital, generate
from oracle.unifloat import map_u32_to_unifloat_bits
from synth import cp_shifts, lattice_vector, nus_seeds, pick, sobol_direction_init

pytestmark = pytest.mark.gpu

XOR = generate.SHIFT_XOR
BACK = generate.LATTICE_BACKWARD


def _mats(s):
    return digital.sobol_matrices(s, sobol_direction_init(s, 0))


def _run_sobol(q, s, first, n, nus, shift, flags=0, ld=None, want_u32=True, want_f32=True):
    import torch

    mats = _mats(s)
    dm = q.from_u32(mats)
    ds = q.from_u32(nus_seeds(s, 1)) if nus else None
    dh = q.from_u32(cp_shifts(s, 2)) if shift else None
    u, f = q.qmc_generate_sobol(dm, first, n, ds, dh, flags, ld=ld, want_u32=want_u32, want_f32=want_f32)
    torch.cuda.synchronize()
    ld = n if ld is None else ld
    gu = q.to_u32(u)[:, :n] if u is not None else None
    gf = f.cpu().numpy()[:, :n].view(np.uint32) if f is not None else None
    eu, ef = generate.generate_sobol(mats, first, n, nus_seeds(s, 1) if nus else None,
                                     cp_shifts(s, 2) if shift else None, flags)
    return gu, gf, eu, ef.view(np.uint32)


SOBOL_CASES = [
    # s, first, n, nus, shift, flags, ld
    (4, 0, 1 << 16, False, False, 0, None),               # unscrambled (0,2)-sequence + 2 dims
    (32, 0, 3 * 2048 + 77, True, True, 0, None),          # several wave runs and a ragged tail
    (32, 4 * 12345, 70001, True, True, XOR, None),        # aligned start, not on a 256 boundary
    (7, 1001, 5000, True, True, 0, None),                 # unaligned start: general kernel
    (5, 0, 100, False, True, 0, None),                    # shift only
    (6, 64, 999, True, False, 0, None),                   # scramble only
    (64, (1 << 32) - 5000, 5000, True, True, 0, None),    # the end of the 32-bit index range
    (9, 256, 3000, True, True, 0, 3004),                  # ld > n, aligned
    (9, 256, 3000, True, True, XOR, 3001),                # odd ld: general kernel
    (3, 12, 1, True, True, 0, None),                      # a single point
]


@pytest.mark.parametrize("case", SOBOL_CASES, ids=[str(c[:3]) for c in SOBOL_CASES])
def test_sobol_bit_exact(qmc, case):
    s, first, n, nus, shift, flags, ld = case
    gu, gf, eu, ef = _run_sobol(qmc, s, first, n, nus, shift, flags, ld)
    assert np.array_equal(gu, eu)
    assert np.array_equal(gf, ef)


def test_sobol_single_output_variants(qmc):
    gu, gf, eu, ef = _run_sobol(qmc, 8, 0, 4096 + 3, True, True, want_f32=False)
    assert gf is None and np.array_equal(gu, eu)
    gu, gf, eu, ef = _run_sobol(qmc, 8, 0, 4096 + 3, True, True, want_u32=False)
    assert gu is None and np.array_equal(gf, ef)


def test_sobol_gpu_output_is_02_net(qmc):
    from test_oracle_digital import net_t_value

    gu, _, _, _ = _run_sobol(qmc, 2, 0, 1 << 16, True, False)
    x, y = gu[0].astype(np.uint64), gu[1].astype(np.uint64)
    for m in range(17):
        nn = 1 << m
        for b in range(min(2, (1 << 16) // nn)):
            sl = slice(b * nn, (b + 1) * nn)
            assert net_t_value(x[sl], y[sl], m) == 0, (m, b)


def _run_lattice(q, s, bits, first, n, shift, flags=0, ld=None):
    import torch

    g = lattice_vector(s, bits, 3)
    dh = q.from_u32(cp_shifts(s, 2)) if shift else None
    u, f = q.qmc_generate_lattice(q.from_u32(g), first, n, dh, flags, ld=ld)
    torch.cuda.synchronize()
    eu, ef = generate.generate_lattice(g, first, n, cp_shifts(s, 2) if shift else None, flags)
    return q.to_u32(u)[:, :n], f.cpu().numpy()[:, :n].view(np.uint32), eu, ef.view(np.uint32)


LATTICE_CASES = [
    (32, 20, 0, 1 << 20, False, 0, None),        # rank-1 lattice sequence n = 2^20, s = 32
    (32, 20, 0, 1 << 20, True, 0, None),         # with an integer Cranley-Patterson rotation
    (16, 30, 4 * 777, 100003, True, XOR, None),
    (16, 30, 0, 70000, False, BACK, None),       # backward enumeration
    (5, 20, (1 << 32) - 4099, 4099, True, BACK, None),
    (7, 20, 3, 5000, True, 0, None),             # unaligned: general kernel
    (7, 20, 8, 5000, True, BACK | XOR, 5003),
]


@pytest.mark.parametrize("case", LATTICE_CASES, ids=[str(c[:4]) for c in LATTICE_CASES])
def test_lattice_bit_exact(qmc, case):
    s, bits, first, n, shift, flags, ld = case
    gu, gf, eu, ef = _run_lattice(qmc, s, bits, first, n, shift, flags, ld)
    assert np.array_equal(gu, eu)
    assert np.array_equal(gf, ef)


def test_lattice_backward_origin_last(qmc):
    gu, gf, _, _ = _run_lattice(qmc, 4, 20, (1 << 32) - 4, 4, False, BACK)
    assert np.all(gu[:, -1] == 0) and np.all(gf[:, -1] == 0)


def test_full_size_scrambled_sobol_sampled(qmc):
    """2^24 points x 32 dims, scramble + rotation, in the benchmark's launch configuration;
    compared on 2^15 random (i, j) samples plus the first and last 1024 indices of every dim."""
    import torch

    s, n = 32, 1 << 24
    mats = _mats(s)
    seeds, shifts = nus_seeds(s, 1), cp_shifts(s, 2)
    u, f = qmc.qmc_generate_sobol(qmc.from_u32(mats), 0, n, qmc.from_u32(seeds), qmc.from_u32(shifts), 0)
    flat = pick(s * n, 1 << 15, 31)
    jj, ii = flat // n, flat % n
    edges = np.concatenate([np.arange(1024), np.arange(n - 1024, n)])
    sel_i = torch.from_numpy(np.concatenate([ii, np.tile(edges, s)])).cuda()
    sel_j = torch.from_numpy(np.concatenate([jj, np.repeat(np.arange(s), edges.size)])).cuda()
    gu = u[sel_j, sel_i].cpu().numpy().view(np.uint32)
    gf = f[sel_j, sel_i].cpu().numpy().view(np.uint32)
    torch.cuda.synchronize()
    si, sj = sel_i.cpu().numpy(), sel_j.cpu().numpy()
    want = np.zeros(si.size, np.uint32)
    for j in range(s):
        m = sj == j
        want[m] = generate.sobol_at(mats, si[m], seeds, shifts, 0, dims=[j])[0]
    assert np.array_equal(gu, want)
    assert np.array_equal(gf, map_u32_to_unifloat_bits(want))
    del u, f


def test_map_u32_to_unifloat_exhaustive(qmc):
    """All 2^32 inputs, as in the paper's own check of the conversion (Sec. 2.1)."""
    import multiprocessing as mp
    from multiprocessing import shared_memory

    import torch

    chunk = 1 << 27
    workers = min(16, os.cpu_count() or 1)
    ctx = mp.get_context("spawn")
    shm = shared_memory.SharedMemory(create=True, size=chunk * 4)
    host = np.ndarray((chunk,), dtype=np.uint32, buffer=shm.buf)
    try:
        with ctx.Pool(workers) as pool:
            for start in range(0, 1 << 32, chunk):
                base = torch.arange(start, start + chunk, dtype=torch.int64, device="cuda")
                inp = torch.where(base >= (1 << 31), base - (1 << 32), base).to(torch.int32)
                out = qmc.qmc_map_u32_to_unifloat(inp)
                host[:] = out.view(torch.int32).cpu().numpy().view(np.uint32)
                step = chunk // workers
                jobs = [(shm.name, chunk, start, k * step, chunk if k == workers - 1 else (k + 1) * step)
                        for k in range(workers)]
                for nbad, first_bad in pool.map(compare_slice, jobs):
                    assert nbad == 0, "mismatch at u=0x%08x" % first_bad
                assert float(out.max()) < 1.0
    finally:
        del host
        shm.close()
        shm.unlink()


def test_argument_errors(qmc):
    import torch

    dm = qmc.from_u32(_mats(4))
    with pytest.raises(qmc.QMCError) as e:
        qmc.qmc_generate_sobol(dm, (1 << 32) - 10, 11)
    assert e.value.status == 2
    with pytest.raises(qmc.QMCError) as e:
        qmc.qmc_generate_sobol(dm, 0, 100, flags=8)
    assert e.value.status == 1
    out = torch.empty((4, 100), dtype=torch.float32, device="cuda")
    with pytest.raises(qmc.QMCError) as e:
        qmc.qmc_generate_sobol(dm, 0, 100, out_u32=out.view(torch.int32), out_f32=out)
    assert e.value.status == 1
    big = qmc.from_u32(np.zeros((65, 32), np.uint32))
    with pytest.raises(qmc.QMCError) as e:
        qmc.qmc_generate_sobol(big, 0, 10)
    assert e.value.status == 2


@pytest.mark.parametrize("cpw,nt", [(1, 0), (3, 1), (8, 0)])
def test_launch_shapes_bit_exact(qmc, cpw, nt, tmp_path):
    """Every launch shape (chunks per wavefront, store kind; set through a tuning file) gives the
    oracle's points, including starts that are not multiples of 256 and the top of the index range."""
    import json

    import torch

    f = tmp_path / "tune.json"
    cfg = {"chunks_per_wave": cpw, "nontemporal": nt}
    f.write_text(json.dumps({"sobol": cfg, "lattice": cfg, "integrate": []}))
    saved = tmp_path / "saved.json"
    qmc.qmc_tune_save(str(saved))
    try:
        qmc.qmc_tune_load(str(f))
        for s, first, n, flags in ((16, 0, 64 * 256 * 5 + 33, 0), (9, 4 * 999, 100001, XOR),
                                   (3, (1 << 32) - 4 * 25001, 100001, 0), (2, 256 * 7, 255, XOR)):
            gu, gf, eu, ef = _run_sobol(qmc, s, first, n, True, True, flags)
            assert np.array_equal(gu, eu) and np.array_equal(gf, ef), (cpw, s, first, n)
            lu, lf, leu, lef = _run_lattice(qmc, s, 30, first, n, True, flags | BACK)
            assert np.array_equal(lu, leu) and np.array_equal(lf, lef), (cpw, s, first, n)
    finally:
        qmc.qmc_tune_load(str(saved))
    torch.cuda.synchronize()


def test_autotune_generate_reports_candidates(qmc):
    mats = qmc.from_u32(_mats(8))
    rep = qmc.qmc_autotune_generate(qmc.QMC_SAMPLER_SOBOL, mats, 1 << 18, qmc.from_u32(nus_seeds(8, 1)),
                                    qmc.from_u32(cp_shifts(8, 2)))
    lines = [l for l in rep.splitlines() if l.strip()]
    assert len(lines) == 8 and all('"ms"' in l for l in lines)
    gu, gf, eu, ef = _run_sobol(qmc, 8, 0, 70000, True, True)
    assert np.array_equal(gu, eu) and np.array_equal(gf, ef)


@pytest.mark.parametrize("kind,s,first,n,flags,ld", [
    ("sobol", 32, 0, 5000, 0, None),
    ("sobol", 7, 4 * 33, 1001, XOR, 9),
    ("sobol", 64, (1 << 32) - 300, 300, 0, None),
    ("sobol", 40, 64 * 1000, 3000, XOR, 45),     # start on a multiple of 64: split index product
    ("sobol", 3, (1 << 32) - 64 * 40, 64 * 40, 0, None),
    ("lattice", 32, 0, 5000, BACK, None),
    ("lattice", 5, 13, 777, XOR, 8),
    ("lattice", 40, 64 * 3, 3000, XOR, 41),     # two groups of dimensions
    ("sobol", 40, 64 * 5, 2000, XOR, 44),       # 16-byte rows: vector stores, then a group of 8
    ("lattice", 36, 0, 1500, XOR, 36),
    # multiples of 32 dimensions with 16-byte rows
    ("sobol", 64, 64 * 77, 4133, XOR, 68),       # two chunks, ragged last tile, gaps between rows
    ("sobol", 32, (1 << 32) - 64 * 50, 64 * 50, 0, 36),   # top of the index range
    ("lattice", 64, 5, 4133, XOR | BACK, 64),
])
def test_point_major_layout(qmc, kind, s, first, n, flags, ld):
    """out[(i - first) * ld + j] against the oracle, bit for bit, and nothing written between
    rows when ld > s."""
    import torch

    pm = qmc.QMC_POINT_MAJOR
    ldv = s if ld is None else ld
    out_u = torch.full((n, ldv), 7, dtype=torch.int32, device="cuda")
    out_f = torch.full((n, ldv), 2.0, dtype=torch.float32, device="cuda")
    if kind == "sobol":
        m = _mats(s)
        qmc.qmc_generate_sobol(qmc.from_u32(m), first, n, qmc.from_u32(nus_seeds(s, 1)), qmc.from_u32(cp_shifts(s, 2)),
                               flags | pm, out_u32=out_u, out_f32=out_f, ld=ldv)
        eu, ef = generate.generate_sobol(m, first, n, nus_seeds(s, 1), cp_shifts(s, 2), flags)
    else:
        g = lattice_vector(s, 20, 3)
        qmc.qmc_generate_lattice(qmc.from_u32(g), first, n, qmc.from_u32(cp_shifts(s, 2)), flags | pm, out_u32=out_u,
                                 out_f32=out_f, ld=ldv)
        eu, ef = generate.generate_lattice(g, first, n, cp_shifts(s, 2), flags)
    torch.cuda.synchronize()
    gu = qmc.to_u32(out_u)
    gf = out_f.cpu().numpy().view(np.uint32)
    assert np.array_equal(gu[:, :s], eu.T)
    assert np.array_equal(gf[:, :s], ef.view(np.uint32).T)
    if ldv > s:
        assert (gu[:, s:] == 7).all() and (out_f[:, s:] == 2.0).all().item()


@pytest.mark.parametrize("s", [33, 64])
def test_point_major_many_tiles_per_wavefront(qmc, s):
    """More 64-point tiles than wavefronts (each wavefront loops over several, unevenly) with two
    groups of dimensions (s = 33: 4-byte stores for the second; s = 64: 16-byte stores for both):
    3000 sampled points against the oracle, whole rows, for the Sobol' and the lattice
    generator."""
    import torch

    first, n = 64 * 7, (1 << 21) + 37
    m = _mats(s)
    seeds, shifts = nus_seeds(s, 1), cp_shifts(s, 2)
    out_u = torch.empty((n, s), dtype=torch.int32, device="cuda")
    qmc.qmc_generate_sobol(qmc.from_u32(m), first, n, qmc.from_u32(seeds), qmc.from_u32(shifts),
                           qmc.QMC_POINT_MAJOR, out_u32=out_u, ld=s)
    rows = np.sort(np.random.default_rng(12).choice(n, 3000, replace=False))
    rows[-1] = n - 1
    got = qmc.to_u32(out_u[torch.from_numpy(rows).cuda()])
    want = generate.sobol_at(m, first + rows.astype(np.uint64), seeds, shifts, 0)
    assert np.array_equal(got, want.T)
    g = lattice_vector(s, 20, 3)
    qmc.qmc_generate_lattice(qmc.from_u32(g), first, n, qmc.from_u32(shifts), qmc.QMC_POINT_MAJOR | BACK,
                             out_u32=out_u, ld=s)
    got = qmc.to_u32(out_u[torch.from_numpy(rows).cuda()])
    want = generate.lattice_at(g, first + rows.astype(np.uint64), shifts, BACK)
    assert np.array_equal(got, want.T)
