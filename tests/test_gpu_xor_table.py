"""GPU parity of the table-driven per-pixel samplers of Sec. 2.6.1.  The XOR sampler:
materialised samples bit for bit against the oracle, the fused forward, adjoint and L2 step
against FP64, a 1920x1080 frame at sampled pixels, and argument errors.  Images wider or taller
than 128 pixels make the tables repeat; sample counts above N make the stored points repeat;
reorder entries span all 32 bits, so the index is reduced modulo N.  The table of
two-dimensional rotations: the same checks for lattice and Sobol' samplers."""

import numpy as np
import pytest

from oracle import digital, estimator, scramble
from synth import (counts_uniform, genz_params, lattice_vector, lobe_params, nus_seeds, perturb, pick,
                   sobol_direction_init, u32_draws)

pytestmark = pytest.mark.gpu

CELLS = 16384


def _est_tol(got, ref):
    env = np.maximum(np.abs(ref["mean"]), ref["env"])
    floor = 1e-6 * max(float(np.max(ref["env"])), 1e-300)
    return np.abs(got.astype(np.float64) - ref["mean"]) <= 2e-5 * np.maximum(env, floor)


def _counts_edge(P):
    base = np.array([0, 1, 2, 3, 63, 64, 65, 127, 128, 129, 200, 256, 5, 31, 32, 33, 1000], dtype=np.uint32)
    return np.resize(base, P)


def _stored_points(s, N, seed):
    """N Owen-scrambled (nested uniform scramble) Sobol' points, u32 [s][N]."""
    mats = digital.sobol_matrices(s, sobol_direction_init(s, 0))
    seeds = nus_seeds(s, seed)
    return np.stack([scramble.nested_uniform_scramble(digital.digital_point(mats[j], np.arange(N, dtype=np.uint64)),
                                                      int(seeds[j])) for j in range(s)]).astype(np.uint32)


def _pair(q, s, N, seed, W):
    import torch

    pts = _stored_points(s, N, seed)
    scr = u32_draws(seed + 100, s * CELLS).reshape(s, CELLS)
    reo = u32_draws(seed + 200, CELLS)
    dev = q.PixelSampler.xor_table(q.from_u32(pts), q.from_u32(scr), q.from_u32(reo))
    ora = {"kind": "xor_table", "s": s, "table": pts, "scramble": scr, "reorder": reo, "width": W}
    return dev, ora


def _all_pairs(counts):
    c = counts.astype(np.int64)
    return np.repeat(np.arange(c.size), c), np.concatenate([np.arange(n) for n in c])


@pytest.mark.parametrize("W,H,d,N", [(131, 4, 8, 256), (6, 130, 40, 64), (129, 2, 3, 1)])
def test_materialised_samples_bit_exact(qmc, W, H, d, N):
    import torch

    P = W * H
    counts = _counts_edge(P)
    ds, os_ = _pair(qmc, d, N, 3, W)
    dc = torch.from_numpy(counts.view(np.int32)).cuda()
    offs = qmc.qmc_sample_offsets(dc)
    total = int(counts.astype(np.int64).sum())
    pts = qmc.qmc_generate_pixel_samples(ds, d, W, H, dc, offs, total)
    torch.cuda.synchronize()
    p_arr, i_arr = _all_pairs(counts)
    want = estimator.pixel_samples_f32(os_, p_arr, i_arr)
    assert np.array_equal(pts.cpu().numpy().view(np.uint32), want.view(np.uint32))


def _genz(q, sampler, W, H, counts, pp):
    import torch

    ig = q.PixelIntegrand.genz(torch.from_numpy(pp).cuda())
    dc = torch.from_numpy(counts.view(np.int32)).cuda()
    m = q.qmc_integrate_pixels(sampler, ig, W, H, dc)
    torch.cuda.synchronize()
    return m.cpu().numpy()


def test_genz_forward_and_plain_equals_fused(qmc):
    import torch

    W, H = 131, 4
    P = W * H
    counts = _counts_edge(P)
    ds, os_ = _pair(qmc, 8, 256, 5, W)
    pp = genz_params(P, 4)
    got = _genz(qmc, ds, W, H, counts, pp)
    ref = estimator.integrate_pixels(os_, {"kind": "genz", "d": 8, "pixel_params": pp}, counts, range(P))
    ok = _est_tol(got, ref)
    assert ok.all(), (np.nonzero(~ok)[0][:10], got[~ok][:5], ref["mean"][~ok][:5])
    dc = torch.from_numpy(counts.view(np.int32)).cuda()
    offs = qmc.qmc_sample_offsets(dc)
    pts = qmc.qmc_generate_pixel_samples(ds, 8, W, H, dc, offs, int(counts.astype(np.int64).sum()))
    plain = _genz(qmc, qmc.PixelSampler.points(pts, offs), W, H, counts, pp)
    assert np.array_equal(got.view(np.uint32), plain.view(np.uint32))


@pytest.mark.parametrize("N", [256, 2])
@pytest.mark.parametrize("begin,end", [(3, 200), (1, 2), (5, 9), (64, 1000), (6, 2**32 - 1)])
def test_genz_sample_windows(qmc, N, begin, end):
    """Windows [begin, end) whose start is not a multiple of four: the fused kernel reads the stored
    points of an aligned group of four samples at once (N >= 4) and takes the samples before the
    first group, and after the last, one at a time; N = 2 takes every sample one at a time.  The
    plain path over the materialised samples of the same window equals the fused one bit for bit
    (pixels with 64 or more samples in the window read a lane per sample, the others a lane per
    pixel)."""
    import torch

    W, H = 131, 4
    P = W * H
    counts = _counts_edge(P)
    ds, os_ = _pair(qmc, 8, N, 5, W)
    pp = genz_params(P, 4)
    ig = qmc.PixelIntegrand.genz(torch.from_numpy(pp).cuda())
    dc = torch.from_numpy(counts.view(np.int32)).cuda()
    got = qmc.qmc_integrate_pixels(ds, ig, W, H, dc, begin, end)
    offs = qmc.qmc_sample_offsets(dc)
    pts = qmc.qmc_generate_pixel_samples(ds, 8, W, H, dc, offs, int(counts.astype(np.int64).sum()))
    plain = qmc.qmc_integrate_pixels(qmc.PixelSampler.points(pts, offs), ig, W, H, dc, begin, end)
    torch.cuda.synchronize()
    got, plain = got.cpu().numpy(), plain.cpu().numpy()
    ref = estimator.integrate_pixels(os_, {"kind": "genz", "d": 8, "pixel_params": pp}, counts, range(P), begin, end)
    ok = _est_tol(got, ref)
    assert ok.all(), (np.nonzero(~ok)[0][:10], got[~ok][:5], ref["mean"][~ok][:5])
    assert np.array_equal(got.view(np.uint32), plain.view(np.uint32))


@pytest.mark.parametrize("d,L,W,H,N", [(8, 64, 131, 2, 128), (40, 7, 3, 130, 64)])
def test_lobes_forward(qmc, d, L, W, H, N):
    import torch

    P = W * H
    counts = _counts_edge(P)
    theta = lobe_params(L, d, 6)
    ds, os_ = _pair(qmc, d, N, 7, W)
    ig = qmc.PixelIntegrand.lobes(torch.from_numpy(theta).cuda(), L, d, 9)
    got = qmc.qmc_integrate_pixels(ds, ig, W, H, torch.from_numpy(counts.view(np.int32)).cuda()).cpu().numpy()
    ref = estimator.integrate_pixels(os_, {"kind": "lobes", "d": d, "num_lobes": L, "params": theta,
                                           "pixel_seed": 9}, counts, range(P))
    assert _est_tol(got, ref).all()


@pytest.mark.parametrize("d,L,W,H", [(8, 64, 131, 2), (64, 32, 5, 2)])
def test_adjoint_and_l2_step(qmc, d, L, W, H):
    """dL/dtheta of the adjoint and of the fused L2 step against the FP64 analytic gradient."""
    import torch

    P = W * H
    counts = counts_uniform(W, H, 64) if d == 64 else _counts_edge(P)
    theta = lobe_params(L, d, 6)
    ds, os_ = _pair(qmc, d, 128, 11, W)
    ig = qmc.PixelIntegrand.lobes(torch.from_numpy(theta).cuda(), L, d, 9)
    oig = {"kind": "lobes", "d": d, "num_lobes": L, "params": theta, "pixel_seed": 9}
    target = estimator.integrate_pixels(os_, dict(oig, params=perturb(theta, 7)), counts, range(P))["mean"]
    loss64, g64, means64 = estimator.loss_and_gradient(os_, oig, counts, range(P), target)
    dc = torch.from_numpy(counts.view(np.int32)).cuda()
    gm = (2.0 * (means64 - target) / P).astype(np.float32)
    g = qmc.qmc_integrate_pixels_backward(ds, ig, W, H, dc, torch.from_numpy(gm).cuda())
    means, loss, g2 = qmc.qmc_integrate_pixels_l2_step(ds, ig, W, H, dc,
                                                       torch.from_numpy(target.astype(np.float32)).cuda())
    torch.cuda.synchronize()
    scale = np.max(np.abs(g64))
    for got in (g.cpu().numpy().astype(np.float64), g2.cpu().numpy().astype(np.float64)):
        ok = np.abs(got - g64) <= 1e-4 * np.maximum(np.abs(g64), 1e-3 * scale)
        assert ok.all(), (np.nonzero(~ok)[0][:10], got[~ok][:5], g64[~ok][:5])
    assert abs(float(loss.cpu()[0]) - loss64) <= 1e-4 * loss64


def test_full_size_genz_sampled_pixels(qmc):
    """1920x1080 x 64 spp from 4096 stored 8-dimensional points; 800 sampled pixels vs FP64."""
    W, H = 1920, 1080
    P = W * H
    counts = counts_uniform(W, H, 64)
    ds, os_ = _pair(qmc, 8, 4096, 13, W)
    pp = genz_params(P, 4)
    got = _genz(qmc, ds, W, H, counts, pp)
    pix = pick(P, 800, 47)
    ref = estimator.integrate_pixels(os_, {"kind": "genz", "d": 8, "pixel_params": pp}, counts, pix)
    ok = _est_tol(got[pix], ref)
    assert ok.all(), (pix[~ok][:10], got[pix][~ok][:5], ref["mean"][~ok][:5])


def test_argument_errors(qmc):
    import torch

    s, N = 8, 64
    pts = qmc.from_u32(_stored_points(s, N, 1))
    scr = qmc.from_u32(u32_draws(1, s * CELLS).reshape(s, CELLS))
    reo = qmc.from_u32(u32_draws(2, CELLS))
    ig = qmc.PixelIntegrand.genz(torch.from_numpy(genz_params(16, 4)).cuda())
    dc = torch.full((16,), 8, dtype=torch.int32, device="cuda")

    def status(sampler):
        with pytest.raises(qmc.QMCError) as e:
            qmc.qmc_integrate_pixels(sampler, ig, 4, 4, dc)
        return e.value.status

    X = qmc.QMC_SAMPLER_XOR_TABLE
    assert status(qmc.PixelSampler(X, pts, 0, qmc.QMC_PIXEL_SHIFT, N, None, s, scr, reo)) == 1   # no flags
    assert status(qmc.PixelSampler(X, pts, 0, 0, 48, None, s, scr, reo)) == 1                   # N not 2^k
    assert status(qmc.PixelSampler(X, pts, 0, 0, 0, None, s, scr, reo)) == 1
    assert status(qmc.PixelSampler(X, pts, 0, 0, N, None, s, None, reo)) == 1                    # no tables
    assert status(qmc.PixelSampler(X, pts, 0, 0, N, None, s, scr, None)) == 1
    with pytest.raises(ValueError):
        qmc.PixelSampler.xor_table(pts[:, :48].contiguous(), scr, reo)
    with pytest.raises(ValueError):
        qmc.PixelSampler.xor_table(pts, scr[:, :100].contiguous(), reo)
    ok = qmc.qmc_integrate_pixels(qmc.PixelSampler.xor_table(pts, scr, reo), ig, 4, 4, dc)
    torch.cuda.synchronize()
    assert ok.shape == (16,)


NUS, SHIFT, XOR, BACK = 4, 8, 1, 2


def _rot_pair(q, kind, s, W, H, flags, seed):
    table = u32_draws(seed, 2 * CELLS).reshape(2, CELLS)
    if kind == "lattice":
        g = lattice_vector(s, 30, 3)
        dev = q.PixelSampler.lattice(q.from_u32(g), 0x51, flags, shift_table=q.from_u32(table))
    else:
        g = digital.sobol_matrices(s, sobol_direction_init(s, 0))
        dev = q.PixelSampler.sobol(q.from_u32(g), 0x51, flags, shift_table=q.from_u32(table))
    ora = {"kind": kind, "s": s, "table": g, "seed": 0x51, "width": W, "height": H, "shift_table": table,
           "flags": flags | SHIFT | estimator.PIXEL_TABLE_SHIFT}
    return dev, ora


ROT_CASES = [
    # kind, flags, W, H, d
    ("lattice", SHIFT, 131, 3, 8),
    ("lattice", SHIFT | XOR | BACK, 5, 130, 40),
    ("sobol", NUS | SHIFT, 131, 3, 8),
    ("sobol", SHIFT | XOR, 4, 131, 3),
]


@pytest.mark.parametrize("case", ROT_CASES, ids=[str(c) for c in ROT_CASES])
def test_table_rotations_materialised_bit_exact(qmc, case):
    import torch

    kind, flags, W, H, d = case
    counts = _counts_edge(W * H)
    ds, os_ = _rot_pair(qmc, kind, d, W, H, flags, 70)
    dc = torch.from_numpy(counts.view(np.int32)).cuda()
    offs = qmc.qmc_sample_offsets(dc)
    pts = qmc.qmc_generate_pixel_samples(ds, d, W, H, dc, offs, int(counts.astype(np.int64).sum()))
    torch.cuda.synchronize()
    p_arr, i_arr = _all_pairs(counts)
    want = estimator.pixel_samples_f32(os_, p_arr, i_arr)
    assert np.array_equal(pts.cpu().numpy().view(np.uint32), want.view(np.uint32))


@pytest.mark.parametrize("kind,flags", [("lattice", SHIFT), ("sobol", NUS | SHIFT)])
def test_table_rotations_fused_genz_and_adjoint(qmc, kind, flags):
    import torch

    W, H = 131, 4
    P = W * H
    counts = _counts_edge(P)
    ds, os_ = _rot_pair(qmc, kind, 8, W, H, flags, 71)
    pp = genz_params(P, 4)
    got = _genz(qmc, ds, W, H, counts, pp)
    ref = estimator.integrate_pixels(os_, {"kind": "genz", "d": 8, "pixel_params": pp}, counts, range(P))
    assert _est_tol(got, ref).all()
    L, d = 64, 8
    theta = lobe_params(L, d, 6)
    ig = qmc.PixelIntegrand.lobes(torch.from_numpy(theta).cuda(), L, d, 9)
    oig = {"kind": "lobes", "d": d, "num_lobes": L, "params": theta, "pixel_seed": 9}
    target = estimator.integrate_pixels(os_, dict(oig, params=perturb(theta, 7)), counts, range(P))["mean"]
    _, g64, means64 = estimator.loss_and_gradient(os_, oig, counts, range(P), target)
    gm = (2.0 * (means64 - target) / P).astype(np.float32)
    g = qmc.qmc_integrate_pixels_backward(ds, ig, W, H, torch.from_numpy(counts.view(np.int32)).cuda(),
                                          torch.from_numpy(gm).cuda())
    torch.cuda.synchronize()
    g = g.cpu().numpy().astype(np.float64)
    ok = np.abs(g - g64) <= 1e-4 * np.maximum(np.abs(g64), 1e-3 * np.max(np.abs(g64)))
    assert ok.all(), (np.nonzero(~ok)[0][:10], g[~ok][:5], g64[~ok][:5])


def test_table_rotation_argument_errors(qmc):
    import torch

    g = qmc.from_u32(lattice_vector(8, 30, 3))
    table = qmc.from_u32(u32_draws(72, 2 * CELLS).reshape(2, CELLS))
    ig = qmc.PixelIntegrand.genz(torch.from_numpy(genz_params(16, 4)).cuda())
    dc = torch.full((16,), 8, dtype=torch.int32, device="cuda")
    L, T = qmc.QMC_SAMPLER_LATTICE, qmc.QMC_PIXEL_TABLE_SHIFT
    for smp in (qmc.PixelSampler(L, g, 1, T, shift_table=table),          # without QMC_PIXEL_SHIFT
                qmc.PixelSampler(L, g, 1, T | SHIFT)):                     # without the table
        with pytest.raises(qmc.QMCError) as e:
            qmc.qmc_integrate_pixels(smp, ig, 4, 4, dc)
        assert e.value.status == 1
    with pytest.raises(ValueError):
        qmc.PixelSampler.lattice(g, 1, shift_table=table[:, :100].contiguous())
    with pytest.raises(TypeError):
        qmc.PixelSampler.lattice(g, 1, shift_table=table.float())
    with pytest.raises(TypeError):
        qmc.PixelSampler.lattice(g.float(), 1)


def test_progressive_graph_with_table_samplers(qmc):
    """Graph-captured progressive passes equal the eager passes bit for bit under both table
    samplers, and a different table of the same shape (a new device buffer) gets its own graph."""
    import torch

    from synth import counts_progressive

    W, H = 140, 9
    P = W * H
    counts = counts_progressive(W, H, 5, passes=4, spp_per_pass=64)
    dc = torch.from_numpy(counts.view(np.int32)).cuda()
    ig = qmc.PixelIntegrand.genz(torch.from_numpy(genz_params(P, 4)).cuda())
    xs, _ = _pair(qmc, 8, 256, 17, W)
    rot_a, _ = _rot_pair(qmc, "lattice", 8, W, H, SHIFT, 80)
    # the same generator buffer, another table: only the table pointer tells the graphs apart
    rot_b = qmc.PixelSampler.lattice(rot_a.table, 0x51, SHIFT,
                                     shift_table=qmc.from_u32(u32_draws(81, 2 * CELLS).reshape(2, CELLS)))
    results = {}
    for name, smp in (("xor", xs), ("rot_a", rot_a), ("rot_b", rot_b)):
        eager = torch.zeros(P, dtype=torch.float32, device="cuda")
        qmc.qmc_integrate_progressive(smp, ig, W, H, dc, 4, 64, eager, use_graph=False)
        for rep in range(2):
            sums = torch.zeros(P, dtype=torch.float32, device="cuda")
            qmc.qmc_integrate_progressive(smp, ig, W, H, dc, 4, 64, sums, use_graph=True)
            torch.cuda.synchronize()
            assert torch.equal(sums, eager), (name, rep)
        results[name] = eager.cpu().numpy()
    assert not np.array_equal(results["rot_a"], results["rot_b"])
