"""GPU parity of per-pixel integration, the plain path, the adjoint and progressive passes.

Tolerances (derived in the design notes from the FP32 arithmetic of the kernels):
  estimates: |I32 - I64| <= 2e-5 * max(|I64|, env_p, 1e-6 * max_q env_q), where env_p is the
             FP64 mean of the envelope |f| bound (Genz: the Gaussian factor; lobes: f itself);
  gradient vs the oracle's analytic FP64 gradient: |g - g64| <= 1e-4 * max(|g64|, 1e-3 max|g64|);
  gradient vs central finite differences of the FP64 loss: 1e-3 in the same form.
Integer samples are compared bit for bit.
"""

import numpy as np
import pytest

from oracle import digital, estimator
from synth import (counts_pow2, counts_uniform, cp_shifts, genz_params, lattice_vector, lobe_params, perturb, pick,
                   sobol_direction_init)

pytestmark = pytest.mark.gpu

NUS, SHIFT, XOR, BACK = 4, 8, 1, 2


def _est_tol(got, ref):
    env = np.maximum(np.abs(ref["mean"]), ref["env"])
    floor = 1e-6 * max(float(np.max(ref["env"])), 1e-300)
    return np.abs(got.astype(np.float64) - ref["mean"]) <= 2e-5 * np.maximum(env, floor)


def _mats(s):
    return digital.sobol_matrices(s, sobol_direction_init(s, 0))


def _sampler_pair(q, kind, s, seed, flags):
    if kind == "sobol":
        m = _mats(s)
        return q.PixelSampler.sobol(q.from_u32(m), seed, flags), {"kind": "sobol", "s": s, "table": m,
                                                                  "seed": seed, "flags": flags}
    g = lattice_vector(s, 30, 3)
    return q.PixelSampler.lattice(q.from_u32(g), seed, flags), {"kind": "lattice", "s": s, "table": g,
                                                                "seed": seed, "flags": flags}


def _counts_edge(P):
    base = np.array([0, 1, 2, 3, 63, 64, 65, 127, 128, 129, 200, 256, 5, 31, 32, 33, 1000], dtype=np.uint32)
    return np.resize(base, P)


def _run_genz(q, sampler, W, H, counts, pp, begin=0, end=2**32 - 1, sums=None):
    import torch

    ig = q.PixelIntegrand.genz(torch.from_numpy(pp).cuda())
    dc = torch.from_numpy(counts.view(np.int32)).cuda()
    means = q.qmc_integrate_pixels(sampler, ig, W, H, dc, begin, end, sums=sums,
                                   means=torch.empty(W * H, dtype=torch.float32, device="cuda"))
    torch.cuda.synchronize()
    return means.cpu().numpy()


GENZ_CASES = [
    # kind, flags, W, H, counts, begin, end
    ("sobol", NUS | SHIFT, 48, 20, "pow2", 0, 2**32 - 1),
    ("sobol", NUS | SHIFT | XOR, 37, 11, "edge", 0, 2**32 - 1),     # ragged last tile, all size classes
    ("sobol", 0, 40, 8, "edge", 0, 2**32 - 1),                      # unscrambled
    ("sobol", SHIFT, 40, 8, "edge", 64, 200),                       # window, aligned start
    ("sobol", NUS, 40, 8, "edge", 37, 150),                         # window, unaligned start
    ("lattice", SHIFT, 48, 20, "pow2", 0, 2**32 - 1),
    ("lattice", SHIFT | BACK | XOR, 37, 11, "edge", 0, 2**32 - 1),
]


@pytest.mark.parametrize("case", GENZ_CASES, ids=[f"{c[0]}-{c[1]}-{c[4]}-{c[5]}" for c in GENZ_CASES])
def test_genz_matches_fp64_oracle(qmc, case):
    kind, flags, W, H, cname, begin, end = case
    P = W * H
    counts = counts_pow2(W, H, 5) if cname == "pow2" else _counts_edge(P)
    pp = genz_params(P, 4)
    ds, os_ = _sampler_pair(qmc, kind, 8, 0x1234, flags)
    got = _run_genz(qmc, ds, W, H, counts, pp, begin, end)
    ref = estimator.integrate_pixels(os_, {"kind": "genz", "d": 8, "pixel_params": pp}, counts, range(P), begin, end)
    # a window's mean is (window sum) / N_p
    ok = _est_tol(got, ref)
    assert ok.all(), (np.nonzero(~ok)[0][:10], got[~ok][:5], ref["mean"][~ok][:5])


def _lobes_setup(q, L, d, seed=6):
    import torch

    theta = lobe_params(L, d, seed)
    return theta, torch.from_numpy(theta).cuda()


LOBE_CASES = [
    # d, L, spp/counts, W, H, kind, flags
    (8, 64, "64", 32, 24, "sobol", NUS | SHIFT),
    (8, 64, "edge", 37, 5, "sobol", NUS | SHIFT),
    (8, 3, "edge", 20, 7, "lattice", SHIFT),
    (5, 70, "edge", 21, 4, "sobol", NUS | SHIFT),          # d < 8, more lobes than one group
    (64, 32, "64", 8, 4, "sobol", NUS | SHIFT),            # two 32-dim halves per lobe
    (20, 7, "edge", 9, 3, "lattice", SHIFT | BACK),
    (50, 45, "edge", 7, 5, "sobol", NUS | SHIFT),          # d > 32 (14 unused dims of 64), two lobe groups
    (40, 33, "64", 5, 3, "lattice", SHIFT),                # one lobe in the second group
]


@pytest.mark.parametrize("case", LOBE_CASES, ids=[f"d{c[0]}-L{c[1]}-{c[2]}-{c[5]}" for c in LOBE_CASES])
def test_lobes_forward_matches_fp64_oracle(qmc, case):
    import torch

    d, L, cname, W, H, kind, flags = case
    P = W * H
    counts = counts_uniform(W, H, 64) if cname == "64" else _counts_edge(P)
    theta, dtheta = _lobes_setup(qmc, L, d)
    ds, os_ = _sampler_pair(qmc, kind, max(d, 8), 77, flags)
    ig = qmc.PixelIntegrand.lobes(dtheta, L, d, 5)
    dc = torch.from_numpy(counts.view(np.int32)).cuda()
    got = qmc.qmc_integrate_pixels(ds, ig, W, H, dc).cpu().numpy()
    ref = estimator.integrate_pixels(os_, {"kind": "lobes", "d": d, "num_lobes": L, "params": theta,
                                           "pixel_seed": 5}, counts, range(P))
    ok = _est_tol(got, ref)
    assert ok.all(), (np.nonzero(~ok)[0][:10], got[~ok][:5], ref["mean"][~ok][:5])


@pytest.mark.parametrize("d,L,kind,flags,begin,end", [
    (8, 64, "sobol", NUS | SHIFT, 37, 150),      # window off a multiple of 64: index parts by the matrix
    (64, 32, "sobol", NUS | SHIFT, 37, 150),
    (64, 32, "sobol", NUS | SHIFT, 64, 300),     # on a multiple of 64: per-round index parts
    (64, 32, "lattice", SHIFT | BACK, 3, 200),
    (40, 7, "sobol", NUS, 128, 2**32 - 1),
])
def test_lobes_forward_windows(qmc, d, L, kind, flags, begin, end):
    """Lobe estimates over sample windows (the progressive passes' building block) against the
    oracle's sums over the same samples."""
    import torch

    W, H = 13, 5
    P = W * H
    counts = _counts_edge(P)
    theta, dtheta = _lobes_setup(qmc, L, d)
    ds, os_ = _sampler_pair(qmc, kind, max(d, 8), 77, flags)
    ig = qmc.PixelIntegrand.lobes(dtheta, L, d, 5)
    dc = torch.from_numpy(counts.view(np.int32)).cuda()
    got = qmc.qmc_integrate_pixels(ds, ig, W, H, dc, begin, end).cpu().numpy()
    ref = estimator.integrate_pixels(os_, {"kind": "lobes", "d": d, "num_lobes": L, "params": theta,
                                           "pixel_seed": 5}, counts, range(P), begin, end)
    ok = _est_tol(got, ref)
    assert ok.all(), (np.nonzero(~ok)[0][:10], got[~ok][:5], ref["mean"][~ok][:5])


@pytest.mark.parametrize("kind,flags", [("sobol", NUS | SHIFT), ("lattice", SHIFT | BACK)])
def test_materialised_samples_bit_exact_and_plain_equals_fused(qmc, kind, flags):
    import torch

    W, H, d = 29, 7, 8
    P = W * H
    counts = _counts_edge(P)
    ds, os_ = _sampler_pair(qmc, kind, 8, 99, flags)
    dc = torch.from_numpy(counts.view(np.int32)).cuda()
    offs = qmc.qmc_sample_offsets(dc)
    torch.cuda.synchronize()
    want_off = np.concatenate([[0], np.cumsum(counts.astype(np.int64))])
    assert np.array_equal(offs.cpu().numpy(), want_off)
    total = int(want_off[-1])
    pts = qmc.qmc_generate_pixel_samples(ds, d, W, H, dc, offs, total)
    torch.cuda.synchronize()
    p_arr = np.repeat(np.arange(P), counts.astype(np.int64))
    i_arr = np.concatenate([np.arange(c) for c in counts.astype(np.int64)])
    want = estimator.pixel_samples_f32(os_, p_arr, i_arr)
    assert np.array_equal(pts.cpu().numpy().view(np.uint32), want.view(np.uint32))
    # the plain path (integrate the materialised samples) gives bitwise the fused result
    pp = genz_params(P, 4)
    fused = _run_genz(qmc, ds, W, H, counts, pp)
    plain = _run_genz(qmc, qmc.PixelSampler.points(pts, offs), W, H, counts, pp)
    assert np.array_equal(fused.view(np.uint32), plain.view(np.uint32))


def test_sums_accumulate_and_windows_compose(qmc):
    import torch

    W, H = 16, 8
    P = W * H
    counts = _counts_edge(P)
    pp = genz_params(P, 4)
    ds, os_ = _sampler_pair(qmc, "sobol", 8, 3, NUS | SHIFT)
    sums = torch.zeros(P, dtype=torch.float32, device="cuda")
    for lo, hi in ((0, 64), (64, 128), (128, 2**32 - 1)):
        _run_genz(qmc, ds, W, H, counts, pp, lo, hi, sums=sums)
    ref = estimator.integrate_pixels(os_, {"kind": "genz", "d": 8, "pixel_params": pp}, counts, range(P))
    got = sums.cpu().numpy().astype(np.float64) / np.maximum(counts, 1)
    assert _est_tol(got.astype(np.float32), ref).all()


def test_forward_is_deterministic_across_schedules(qmc):
    import torch

    W, H = 64, 16
    P = W * H
    counts = counts_pow2(W, H, 5)
    pp = genz_params(P, 4)
    ds, _ = _sampler_pair(qmc, "sobol", 8, 5, NUS | SHIFT)
    a = _run_genz(qmc, ds, W, H, counts, pp)
    b = _run_genz(qmc, ds, W, H, counts, pp)
    dc = torch.from_numpy(counts.view(np.int32)).cuda()
    qmc.qmc_autotune_integrate(ds, qmc.PixelIntegrand.genz(torch.from_numpy(pp).cuda()), W, H, dc)
    c = _run_genz(qmc, ds, W, H, counts, pp)
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
    assert np.array_equal(a.view(np.uint32), c.view(np.uint32))


def _grad_case(qmc, d, L, W, H, counts, kind="sobol", flags=NUS | SHIFT):
    import torch

    P = W * H
    theta, dtheta = _lobes_setup(qmc, L, d)
    target_theta = perturb(theta, 7)
    ds, os_ = _sampler_pair(qmc, kind, max(d, 8), 21, flags)
    ig = qmc.PixelIntegrand.lobes(dtheta, L, d, 9)
    oig = {"kind": "lobes", "d": d, "num_lobes": L, "params": theta, "pixel_seed": 9}
    target = estimator.integrate_pixels(os_, dict(oig, params=target_theta), counts, range(P))["mean"]
    loss, g64, means = estimator.loss_and_gradient(os_, oig, counts, range(P), target)
    gm = (2.0 * (means - target) / P).astype(np.float32)
    dc = torch.from_numpy(counts.view(np.int32)).cuda()
    g = qmc.qmc_integrate_pixels_backward(ds, ig, W, H, dc, torch.from_numpy(gm).cuda())
    torch.cuda.synchronize()
    return g.cpu().numpy().astype(np.float64), g64, (os_, oig, counts, target)


@pytest.mark.parametrize("d,L,W,H,cname", [(8, 64, 24, 16, "64"), (8, 64, 23, 5, "edge"), (5, 70, 13, 4, "edge"),
                                           (64, 32, 6, 4, "64"), (20, 7, 9, 3, "edge")])
def test_adjoint_matches_analytic_fp64_gradient(qmc, d, L, W, H, cname):
    counts = counts_uniform(W, H, 64) if cname == "64" else _counts_edge(W * H)
    g, g64, _ = _grad_case(qmc, d, L, W, H, counts)
    scale = np.max(np.abs(g64))
    err = np.abs(g - g64)
    ok = err <= 1e-4 * np.maximum(np.abs(g64), 1e-3 * scale)
    assert ok.all(), (np.nonzero(~ok)[0][:10], g[~ok][:5], g64[~ok][:5])


def test_adjoint_matches_central_differences(qmc):
    W, H, d, L = 16, 12, 8, 64
    counts = counts_uniform(W, H, 64)
    g, g64, (os_, oig, counts, target) = _grad_case(qmc, d, L, W, H, counts)
    idx = pick(L * (2 * d + 1), 16, 8)
    fd = estimator.finite_difference(os_, oig, counts, range(W * H), target, idx)
    scale = np.max(np.abs(fd))
    ok = np.abs(g[idx] - fd) <= 1e-3 * np.maximum(np.abs(fd), 1e-3 * scale)
    assert ok.all(), (idx[~ok], g[idx][~ok], fd[~ok])


def test_adjoint_is_deterministic(qmc):
    W, H = 32, 8
    counts = _counts_edge(W * H)
    g1, _, _ = _grad_case(qmc, 8, 64, W, H, counts)
    g2, _, _ = _grad_case(qmc, 8, 64, W, H, counts)
    assert np.array_equal(g1, g2)


def test_autograd_function(qmc):
    import torch

    W, H, d, L = 16, 8, 8, 16
    P = W * H
    counts = counts_uniform(W, H, 64)
    theta, dtheta = _lobes_setup(qmc, L, d)
    ds, _ = _sampler_pair(qmc, "sobol", 8, 21, NUS | SHIFT)
    ig = qmc.PixelIntegrand.lobes(dtheta, L, d, 9)
    dc = torch.from_numpy(counts.view(np.int32)).cuda()
    th = dtheta.clone().requires_grad_(True)
    target = torch.rand(P, device="cuda")
    means = qmc.integrate(th, ds, ig, W, H, dc)
    loss = ((means - target) ** 2).mean()
    loss.backward()
    gm = (2.0 * (means.detach() - target) / P).contiguous()
    direct = qmc.qmc_integrate_pixels_backward(ds, ig, W, H, dc, gm)
    torch.cuda.synchronize()
    assert torch.equal(th.grad, direct)


def test_progressive_graph_replays_match_eager(qmc):
    import torch

    from synth import counts_progressive

    W, H, d, L = 24, 8, 8, 8
    P = W * H
    counts = counts_progressive(W, H, 5, passes=4, spp_per_pass=64)
    theta, dtheta = _lobes_setup(qmc, L, d)
    ds, os_ = _sampler_pair(qmc, "sobol", 8, 31, NUS | SHIFT)
    ig = qmc.PixelIntegrand.lobes(dtheta, L, d, 2)
    dc = torch.from_numpy(counts.view(np.int32)).cuda()
    eager = torch.zeros(P, dtype=torch.float32, device="cuda")
    qmc.qmc_integrate_progressive(ds, ig, W, H, dc, 4, 64, eager, use_graph=False)
    torch.cuda.synchronize()
    e = eager.cpu().numpy()
    for rep in range(3):  # replays of one cached graph, with eager work in between
        sums = torch.zeros(P, dtype=torch.float32, device="cuda")
        means = torch.zeros(P, dtype=torch.float32, device="cuda")
        qmc.qmc_integrate_progressive(ds, ig, W, H, dc, 4, 64, sums, means, use_graph=True)
        torch.cuda.synchronize()
        assert np.array_equal(sums.cpu().numpy().view(np.uint32), e.view(np.uint32)), rep
        torch.zeros(1 << 20, device="cuda").add_(1.0)
    ref = estimator.integrate_pixels(os_, {"kind": "lobes", "d": d, "num_lobes": L, "params": theta,
                                           "pixel_seed": 2}, counts, range(P))
    assert _est_tol(means.cpu().numpy(), ref).all()


def test_full_size_genz_sampled_pixels(qmc):
    """1920x1080, counts 2^k in [1,256], one persistent launch; 1500 sampled pixels vs FP64."""
    import torch

    W, H = 1920, 1080
    P = W * H
    counts = counts_pow2(W, H, 5)
    pp = genz_params(P, 4)
    ds, os_ = _sampler_pair(qmc, "sobol", 8, 0xC3, NUS | SHIFT)
    got = _run_genz(qmc, ds, W, H, counts, pp)
    pix = pick(P, 1500, 41)
    ref = estimator.integrate_pixels(os_, {"kind": "genz", "d": 8, "pixel_params": pp}, counts, pix)
    ok = _est_tol(got[pix], ref)
    assert ok.all(), (pix[~ok][:10], got[pix][~ok][:5], ref["mean"][~ok][:5])


def test_full_size_lobes_forward_sampled_pixels(qmc):
    """1920x1080 x 64 spp, 64 lobes in 8 dims; 400 sampled pixels vs FP64."""
    import torch

    W, H, d, L = 1920, 1080, 8, 64
    P = W * H
    counts = counts_uniform(W, H, 64)
    theta, dtheta = _lobes_setup(qmc, L, d)
    ds, os_ = _sampler_pair(qmc, "sobol", 8, 0xC4, NUS | SHIFT)
    ig = qmc.PixelIntegrand.lobes(dtheta, L, d, 9)
    dc = torch.from_numpy(counts.view(np.int32)).cuda()
    got = qmc.qmc_integrate_pixels(ds, ig, W, H, dc).cpu().numpy()
    pix = pick(P, 400, 42)
    ref = estimator.integrate_pixels(os_, {"kind": "lobes", "d": d, "num_lobes": L, "params": theta,
                                           "pixel_seed": 9}, counts, pix)
    assert _est_tol(got[pix], ref).all()


@pytest.mark.parametrize("kind,flags", [("sobol", NUS | SHIFT), ("lattice", SHIFT)])
def test_full_size_progressive_sampled_pixels(qmc, kind, flags):
    """The 3840x2160 progressive workload as timed: 16 graph-replayed passes of 64 spp, counts
    64..1024, 32 lobes in 64 dims, Sobol' (NUS + shift) or lattice (shift) samples.  Means at 300
    sampled pixels vs FP64; then (Sobol') the adjoint over the whole frame with dL/dI nonzero
    only at 48 sampled pixels vs the FP64 gradient of those pixels, within 1e-4 relative or 2e-5
    of the size of the terms summed."""
    import torch

    from synth import counts_progressive

    W, H, d, L = 3840, 2160, 64, 32
    P = W * H
    counts = counts_progressive(W, H, 5, passes=16, spp_per_pass=64)
    theta, dtheta = _lobes_setup(qmc, L, d)
    ds, os_ = _sampler_pair(qmc, kind, 64, 0xC5, flags)
    ig = qmc.PixelIntegrand.lobes(dtheta, L, d, 9)
    oig = {"kind": "lobes", "d": d, "num_lobes": L, "params": theta, "pixel_seed": 9}
    dc = torch.from_numpy(counts.view(np.int32)).cuda()
    sums = torch.zeros(P, dtype=torch.float32, device="cuda")
    means = torch.empty(P, dtype=torch.float32, device="cuda")
    qmc.qmc_integrate_progressive(ds, ig, W, H, dc, 16, 64, sums, means, use_graph=True)
    torch.cuda.synchronize()
    pix = pick(P, 300, 44)
    got = means[torch.from_numpy(pix).cuda()].cpu().numpy()
    ref = estimator.integrate_pixels(os_, oig, counts, pix)
    ok = _est_tol(got, ref)
    assert ok.all(), (pix[~ok][:10], got[~ok][:5], ref["mean"][~ok][:5])
    del sums, means
    if kind != "sobol":
        return

    gpix = pick(P, 48, 45)
    gvals = (np.random.default_rng(46).uniform(-1.0, 1.0, gpix.size) / gpix.size).astype(np.float32)
    gm = torch.zeros(P, dtype=torch.float32, device="cuda")
    gm[torch.from_numpy(gpix).cuda()] = torch.from_numpy(gvals).cuda()
    g = qmc.qmc_integrate_pixels_backward(ds, ig, W, H, dc, gm)
    torch.cuda.synchronize()
    g = g.cpu().numpy().astype(np.float64)
    g64 = estimator.lobes_gradient(os_, oig, counts, gpix, gvals)
    size = estimator.lobes_gradient(os_, oig, counts, gpix, gvals, sizes=True)
    err = np.abs(g - g64)
    ok = (err <= 1e-4 * np.abs(g64)) | (err <= 2e-5 * size)
    assert ok.all(), (np.nonzero(~ok)[0][:10], g[~ok][:5], g64[~ok][:5], size[~ok][:5])


def test_integration_argument_errors(qmc):
    import torch

    W, H = 8, 8
    dc = torch.ones(W * H, dtype=torch.int32, device="cuda")
    ds, _ = _sampler_pair(qmc, "sobol", 8, 1, NUS | SHIFT)
    ig = qmc.PixelIntegrand.genz(torch.zeros((W * H, 16), device="cuda"))
    with pytest.raises(qmc.QMCError) as e:
        qmc.qmc_integrate_pixels(ds, ig, W, H, dc, 10, 5)
    assert e.value.status == 1
    with pytest.raises(qmc.QMCError) as e:
        qmc.qmc_integrate_pixels_backward(ds, ig, W, H, dc, torch.zeros(W * H, device="cuda"),
                                          torch.zeros(16, device="cuda"))
    assert e.value.status == 3
    small, _ = _sampler_pair(qmc, "sobol", 4, 1, NUS)
    with pytest.raises(qmc.QMCError) as e:
        qmc.qmc_integrate_pixels(small, ig, W, H, dc)
    assert e.value.status == 1
    lat, _ = _sampler_pair(qmc, "lattice", 8, 1, SHIFT)
    bad = qmc.PixelSampler(qmc.QMC_SAMPLER_LATTICE, lat.table, 1, NUS)
    with pytest.raises(qmc.QMCError) as e:
        qmc.qmc_integrate_pixels(bad, ig, W, H, dc)
    assert e.value.status == 1
    ws = torch.empty(16, dtype=torch.uint8, device="cuda")
    with pytest.raises(qmc.QMCError) as e:
        qmc.qmc_integrate_pixels(ds, ig, W, H, dc, workspace=ws)
    assert e.value.status == 5


@pytest.mark.parametrize("d,L,W,H,cname", [(8, 64, 40, 8, "64"), (8, 64, 23, 5, "edge"), (8, 100, 16, 4, "64"),
                                           (64, 32, 6, 4, "64"), (5, 7, 13, 4, "edge")])
def test_fused_l2_step_matches_oracle(qmc, d, L, W, H, cname):
    """The fused forward + L2 gradient + adjoint kernel: loss, means and dL/dtheta against
    the FP64 oracle: one walk per tile (d <= 8, one lane group) with big pixels only and with
    packed, empty and big pixels mixed, and the two-walk variant (more lobes than lanes, d = 64)."""
    import torch

    P = W * H
    counts = counts_uniform(W, H, 64) if cname == "64" else _counts_edge(P)
    theta, dtheta = _lobes_setup(qmc, L, d)
    ds, os_ = _sampler_pair(qmc, "sobol", max(d, 8), 21, NUS | SHIFT)
    ig = qmc.PixelIntegrand.lobes(dtheta, L, d, 9)
    oig = {"kind": "lobes", "d": d, "num_lobes": L, "params": theta, "pixel_seed": 9}
    target = estimator.integrate_pixels(os_, dict(oig, params=perturb(theta, 7)), counts, range(P))["mean"]
    loss64, g64, means64 = estimator.loss_and_gradient(os_, oig, counts, range(P), target)
    dc = torch.from_numpy(counts.view(np.int32)).cuda()
    means, loss, grad = qmc.qmc_integrate_pixels_l2_step(ds, ig, W, H, dc, torch.from_numpy(target.astype(np.float32)).cuda())
    torch.cuda.synchronize()
    ref = estimator.integrate_pixels(os_, oig, counts, range(P))
    assert _est_tol(means.cpu().numpy(), ref).all()
    g = grad.cpu().numpy().astype(np.float64)
    ok = np.abs(g - g64) <= 1e-4 * np.maximum(np.abs(g64), 1e-3 * np.max(np.abs(g64)))
    assert ok.all(), (np.nonzero(~ok)[0][:10], g[~ok][:5], g64[~ok][:5])
    assert abs(float(loss.cpu()[0]) - loss64) <= 1e-4 * loss64


def test_binding_rejects_bad_plain_path_buffers(qmc):
    """The binding checks dtype and shape of every buffer the sample kernels index through
    device-resident offsets, before any launch."""
    import torch

    W, H, d = 8, 4, 8
    P = W * H
    counts = _counts_edge(P)
    ds, _ = _sampler_pair(qmc, "sobol", 8, 3, NUS | SHIFT)
    dc = torch.from_numpy(counts.view(np.int32)).cuda()
    offs = qmc.qmc_sample_offsets(dc)
    total = int(counts.astype(np.int64).sum())
    with pytest.raises(TypeError):   # int32 offsets
        qmc.qmc_generate_pixel_samples(ds, d, W, H, dc, offs.to(torch.int32), total)
    with pytest.raises(TypeError):   # offsets of the wrong length
        qmc.qmc_generate_pixel_samples(ds, d, W, H, dc, offs[:-1], total)
    with pytest.raises(TypeError):   # float64 output
        qmc.qmc_generate_pixel_samples(ds, d, W, H, dc, offs, total,
                                       out=torch.empty((d, total), dtype=torch.float64, device="cuda"))
    with pytest.raises(ValueError):  # too few rows
        qmc.qmc_generate_pixel_samples(ds, d, W, H, dc, offs, total,
                                       out=torch.empty((d - 1, total), dtype=torch.float32, device="cuda"))
    with pytest.raises(ValueError):  # too few columns
        qmc.qmc_generate_pixel_samples(ds, d, W, H, dc, offs, total,
                                       out=torch.empty((d, total - 1), dtype=torch.float32, device="cuda"))
    pts = qmc.qmc_generate_pixel_samples(ds, d, W, H, dc, offs, total)
    with pytest.raises(TypeError):
        qmc.PixelSampler.points(pts, offs.to(torch.int32))
    with pytest.raises(TypeError):
        qmc.PixelSampler.points(pts.double(), offs)
    ig = qmc.PixelIntegrand.genz(torch.from_numpy(genz_params(P, 4)).cuda())
    short = qmc.PixelSampler.points(pts, offs[:-1])
    with pytest.raises(ValueError):
        qmc.qmc_integrate_pixels(short, ig, W, H, dc)
    torch.cuda.synchronize()


def test_autograd_keeps_the_shape_of_theta(qmc):
    """A parameter tensor of any shape gets a gradient of its own shape (the kernels see the
    flat [L (2d + 1)] layout)."""
    import torch

    W, H, d, L = 8, 8, 8, 4
    counts = counts_uniform(W, H, 64)
    theta, dtheta = _lobes_setup(qmc, L, d)
    ds, _ = _sampler_pair(qmc, "sobol", 8, 21, NUS | SHIFT)
    ig = qmc.PixelIntegrand.lobes(dtheta, L, d, 9)
    dc = torch.from_numpy(counts.view(np.int32)).cuda()
    th = dtheta.clone().view(L, 2 * d + 1).requires_grad_(True)
    means = qmc.integrate(th, ds, ig, W, H, dc)
    means.sum().backward()
    assert th.grad.shape == th.shape
    flat = dtheta.clone().requires_grad_(True)
    qmc.integrate(flat, ds, ig, W, H, dc).sum().backward()
    torch.cuda.synchronize()
    assert torch.equal(th.grad.reshape(-1), flat.grad)


def _confined_grad_ok(g, g64, size):
    """The gradient tolerance: |g - g64| <= 1e-4 max(|g64|, 1e-3 max|g64|); components whose
    summed term sizes exceed five times that scale (they cancel) may instead be within 2e-5 of
    the size of the terms, the FP32 rounding bound of their sums."""
    scale = np.maximum(np.abs(g64), 1e-3 * np.max(np.abs(g64)))
    err = np.abs(g - g64)
    return (err <= 1e-4 * scale) | ((size > 5 * scale) & (err <= 2e-5 * size))


def _c4_setup(qmc):
    """The 1920x1080 x 64 spp lobe workload (d = 8, 64 lobes), in the launch shape the benchmark
    times (the autotuner's choice for the forward and the adjoint direction)."""
    import torch

    W, H, d, L = 1920, 1080, 8, 64
    P = W * H
    counts = counts_uniform(W, H, 64)
    theta, dtheta = _lobes_setup(qmc, L, d)
    ds, os_ = _sampler_pair(qmc, "sobol", 8, 0xC4, NUS | SHIFT)
    ig = qmc.PixelIntegrand.lobes(dtheta, L, d, 9)
    oig = {"kind": "lobes", "d": d, "num_lobes": L, "params": theta, "pixel_seed": 9}
    dc = torch.from_numpy(counts.view(np.int32)).cuda()
    qmc.qmc_autotune_integrate(ds, ig, W, H, dc)
    qmc.qmc_autotune_integrate(ds, ig, W, H, dc, backward=True,
                               grad_means=torch.full((P,), 1e-7, dtype=torch.float32, device="cuda"))
    return W, H, P, counts, dc, ds, os_, ig, oig


def test_full_size_lobes_adjoint_sampled_pixels(qmc):
    """1920x1080 x 64 spp adjoint over the whole frame with dL/dI nonzero at 48 sampled pixels,
    against the FP64 gradient of those pixels."""
    import torch

    W, H, P, counts, dc, ds, os_, ig, oig = _c4_setup(qmc)
    gpix = pick(P, 48, 47)
    gvals = (np.random.default_rng(48).uniform(-1.0, 1.0, gpix.size) / gpix.size).astype(np.float32)
    gm = torch.zeros(P, dtype=torch.float32, device="cuda")
    gm[torch.from_numpy(gpix).cuda()] = torch.from_numpy(gvals).cuda()
    g = qmc.qmc_integrate_pixels_backward(ds, ig, W, H, dc, gm)
    torch.cuda.synchronize()
    g = g.cpu().numpy().astype(np.float64)
    g64 = estimator.lobes_gradient(os_, oig, counts, gpix, gvals)
    size = estimator.lobes_gradient(os_, oig, counts, gpix, gvals, sizes=True)
    ok = _confined_grad_ok(g, g64, size)
    assert ok.all(), (np.nonzero(~ok)[0][:10], g[~ok][:5], g64[~ok][:5], size[~ok][:5])


def test_full_size_fused_l2_step_sampled_pixels(qmc):
    """The fused forward + L2 gradient + adjoint at 1920x1080 x 64 spp.  A first call gives the
    means; the target is set to them except at 48 sampled pixels, so in a second call (bitwise
    the same estimates) dL/dI_p = 2 (I_p - T_p) / P is exactly zero at every other pixel.  Means
    at 400 sampled pixels against FP64, the loss and the gradient against the FP64 values of the
    48 perturbed pixels."""
    import torch

    W, H, P, counts, dc, ds, os_, ig, oig = _c4_setup(qmc)
    zero = torch.zeros(P, dtype=torch.float32, device="cuda")
    m1, _, _ = qmc.qmc_integrate_pixels_l2_step(ds, ig, W, H, dc, zero)
    torch.cuda.synchronize()
    i32 = m1.cpu().numpy()
    gpix = pick(P, 48, 49)
    delta = np.random.default_rng(50).uniform(-0.02, 0.02, gpix.size) * np.abs(i32[gpix])
    target = i32.copy()
    target[gpix] = (i32[gpix].astype(np.float64) - delta).astype(np.float32)
    m2, loss, g = qmc.qmc_integrate_pixels_l2_step(ds, ig, W, H, dc, torch.from_numpy(target).cuda())
    torch.cuda.synchronize()
    assert np.array_equal(m2.cpu().numpy().view(np.uint32), i32.view(np.uint32))
    pix = pick(P, 400, 51)
    ref = estimator.integrate_pixels(os_, oig, counts, pix)
    ok = _est_tol(i32[pix], ref)
    assert ok.all(), (pix[~ok][:10], i32[pix][~ok][:5], ref["mean"][~ok][:5])
    diff = i32[gpix].astype(np.float64) - target[gpix].astype(np.float64)
    loss64 = float(np.sum(diff * diff)) / P
    assert abs(float(loss.cpu()[0]) - loss64) <= 1e-4 * loss64
    gvals = 2.0 * diff / P
    g = g.cpu().numpy().astype(np.float64)
    g64 = estimator.lobes_gradient(os_, oig, counts, gpix, gvals)
    size = estimator.lobes_gradient(os_, oig, counts, gpix, gvals, sizes=True)
    ok = _confined_grad_ok(g, g64, size)
    assert ok.all(), (np.nonzero(~ok)[0][:10], g[~ok][:5], g64[~ok][:5], size[~ok][:5])


@pytest.mark.parametrize("d,L,W,H", [(8, 64, 40, 30), (64, 32, 20, 13)])
def test_adjoint_is_schedule_independent(qmc, d, L, W, H, tmp_path):
    """The adjoint and the fused L2 step give bitwise the same results under every launch shape
    (persistent grid of 1 to 32 wavefronts per compute unit, static or queued): each tile's
    float32 partial is fixed, and the partials are summed exactly, so neither the wavefront that
    runs a tile nor the order of the additions can change a bit."""
    import json

    import torch

    P = W * H
    counts = _counts_edge(P)
    theta, dtheta = _lobes_setup(qmc, L, d)
    ds, _ = _sampler_pair(qmc, "sobol", max(d, 8), 21, NUS | SHIFT)
    ig = qmc.PixelIntegrand.lobes(dtheta, L, d, 9)
    dc = torch.from_numpy(counts.view(np.int32)).cuda()
    gm = torch.from_numpy(np.random.default_rng(3).uniform(-1, 1, P).astype(np.float32) / P).cuda()
    target = torch.from_numpy(np.random.default_rng(4).uniform(0, 1, P).astype(np.float32)).cuda()
    key = (qmc.QMC_F_LOBES << 16) | (d << 1) | 1
    saved = tmp_path / "saved.json"
    qmc.qmc_tune_save(str(saved))
    results = []
    try:
        for w, dyn in ((1, 0), (4, 1), (16, 0), (32, 1)):
            f = tmp_path / ("tune_%d_%d.json" % (w, dyn))
            cfg = {"chunks_per_wave": 1, "nontemporal": 0}
            f.write_text(json.dumps({"sobol": cfg, "lattice": cfg,
                                     "integrate": [{"key": key, "waves_per_cu": w, "dynamic": dyn}]}))
            qmc.qmc_tune_load(str(f))
            g = qmc.qmc_integrate_pixels_backward(ds, ig, W, H, dc, gm)
            _, loss, sg = qmc.qmc_integrate_pixels_l2_step(ds, ig, W, H, dc, target)
            torch.cuda.synchronize()
            results.append([t.cpu().numpy().view(np.uint32) for t in (g, loss, sg)])
    finally:
        qmc.qmc_tune_load(str(saved))
    for r in results[1:]:
        for a, b in zip(results[0], r):
            assert np.array_equal(a, b)


def test_adjoint_workspace_is_bounded(qmc):
    """The adjoint's workspace is its exact accumulator, 640 bytes per gradient entry whatever the
    frame size: 2.6 MB for the 3840x2160 adjoint with 32 lobes in 64 dimensions (4128
    parameters, plus the loss for the L2 step)."""
    import torch

    m = _mats(64)
    ds = qmc.PixelSampler.sobol(qmc.from_u32(m), 1, NUS | SHIFT)
    ig = qmc.PixelIntegrand.lobes(torch.zeros(32 * 129, device="cuda"), 32, 64, 9)
    for mode in (1, 2):
        n_row = 4128 + (mode == 2)
        for W, H in ((3840, 2160), (64, 1)):
            assert qmc.qmc_workspace_size(ds, ig, W, H, mode) == 1024 + 640 * n_row
    ig8 = qmc.PixelIntegrand.lobes(torch.zeros(64 * 17, device="cuda"), 64, 8, 9)
    assert qmc.qmc_workspace_size(ds, ig8, 1920, 1080, 1) == 1024 + 640 * 1088
