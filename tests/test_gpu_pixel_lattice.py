"""GPU parity of the per-pixel lattice samplers of Sec. 3: the per-pixel random generator
(Alg. 4, optionally four superimposed instances) and the Hilbert-curve shift of the radical
inverse (Eq. PixelShiftedR1LS).  Samples are compared bit for bit with the oracle; estimates
to the tolerance of test_gpu_integrate.  Gradient components pass that file's bound or, where
their terms cancel, the FP32 rounding bound 2e-5 * B (B: the summed sizes of the terms,
including dL/dI_p's rounding relative to |I_p|; 2e-5 ~ 256 * 2^-24 for up to 256 sequential
additions per pixel)."""

import numpy as np
import pytest

from oracle import estimator
from synth import counts_pow2, genz_params, lattice_vector, lobe_params, perturb

pytestmark = pytest.mark.gpu

SHIFT, XOR, BACK = 8, 1, 2
RGEN, HIL, INST4 = 16, 32, 64


def _counts(P):
    base = np.array([0, 1, 2, 3, 63, 64, 65, 127, 128, 129, 200, 256, 5, 31, 32, 33, 100], dtype=np.uint32)
    return np.resize(base, P)


def _pair(q, s, seed, flags, W, H):
    g = lattice_vector(s, 30, 3)
    return (q.PixelSampler.lattice(q.from_u32(g), seed, flags),
            {"kind": "lattice", "s": s, "table": g, "seed": seed, "flags": flags, "width": W, "height": H})


def _est_tol(got, ref):
    env = np.maximum(np.abs(ref["mean"]), ref["env"])
    floor = 1e-6 * max(float(np.max(ref["env"])), 1e-300)
    return np.abs(got.astype(np.float64) - ref["mean"]) <= 2e-5 * np.maximum(env, floor)


CASES = [
    # d, W, H, flags
    (8, 19, 7, HIL),
    (8, 19, 7, HIL | SHIFT | XOR),
    (8, 23, 4, RGEN),
    (8, 23, 4, RGEN | INST4 | BACK),
    (8, 11, 9, RGEN | INST4 | HIL | SHIFT),
    (40, 9, 5, HIL | RGEN | BACK),          # d > 32: two lanes share each sample
    (5, 33, 2, RGEN | INST4 | HIL),
]


@pytest.mark.parametrize("d,W,H,flags", CASES)
def test_materialised_samples_bit_exact(qmc, d, W, H, flags):
    import torch

    P = W * H
    counts = _counts(P)
    ds, os_ = _pair(qmc, max(d, 8), 1234, flags, W, H)
    dc = torch.from_numpy(counts.view(np.int32)).cuda()
    offs = qmc.qmc_sample_offsets(dc)
    total = int(counts.astype(np.int64).sum())
    pts = qmc.qmc_generate_pixel_samples(ds, d, W, H, dc, offs, total)
    torch.cuda.synchronize()
    p_arr = np.repeat(np.arange(P), counts.astype(np.int64))
    i_arr = np.concatenate([np.arange(c) for c in counts.astype(np.int64)])
    want = estimator.pixel_samples_f32(os_, p_arr, i_arr)[:d]
    got = pts.cpu().numpy()[:d]
    assert np.array_equal(got.view(np.uint32), want.view(np.uint32)), (d, W, H, flags)


@pytest.mark.parametrize("flags", [HIL | SHIFT, RGEN | INST4 | SHIFT, RGEN | HIL])
def test_genz_estimates_and_windows(qmc, flags):
    import torch

    W, H = 37, 11
    P = W * H
    counts = counts_pow2(W, H, 5)
    pp = genz_params(P, 4)
    ds, os_ = _pair(qmc, 8, 77, flags, W, H)
    ig = qmc.PixelIntegrand.genz(torch.from_numpy(pp).cuda())
    dc = torch.from_numpy(counts.view(np.int32)).cuda()
    means = qmc.qmc_integrate_pixels(ds, ig, W, H, dc)
    torch.cuda.synchronize()
    ref = estimator.integrate_pixels(os_, {"kind": "genz", "d": 8, "pixel_params": pp}, counts, range(P))
    assert _est_tol(means.cpu().numpy(), ref).all()
    # windows [0,64), [64,128), [128, end) sum to the whole (graph-free progressive use)
    sums = torch.zeros(P, dtype=torch.float32, device="cuda")
    for lo, hi in ((0, 64), (64, 128), (128, 2 ** 32 - 1)):
        qmc.qmc_integrate_pixels(ds, ig, W, H, dc, lo, hi, sums=sums)
    torch.cuda.synchronize()
    got = sums.cpu().numpy().astype(np.float64) / np.maximum(counts, 1)
    assert _est_tol(got.astype(np.float32), ref).all()


@pytest.mark.parametrize("flags", [RGEN | INST4 | SHIFT, HIL | BACK])
@pytest.mark.parametrize("begin,end", [(3, 70), (1, 2), (130, 2 ** 32 - 1)])
def test_genz_unaligned_windows(qmc, flags, begin, end):
    """Windows whose first sample is not instance 0 of the four superimposed instances (nor on a
    multiple of 64): window sums against the oracle's over the same samples."""
    import torch

    W, H = 37, 11
    P = W * H
    counts = counts_pow2(W, H, 5)
    pp = genz_params(P, 4)
    ds, os_ = _pair(qmc, 8, 77, flags, W, H)
    ig = qmc.PixelIntegrand.genz(torch.from_numpy(pp).cuda())
    dc = torch.from_numpy(counts.view(np.int32)).cuda()
    means = qmc.qmc_integrate_pixels(ds, ig, W, H, dc, begin, end)
    torch.cuda.synchronize()
    ref = estimator.integrate_pixels(os_, {"kind": "genz", "d": 8, "pixel_params": pp}, counts, range(P), begin, end)
    assert _est_tol(means.cpu().numpy(), ref).all()


@pytest.mark.parametrize("d,L,W,H,cname,flags", [(8, 64, 40, 8, "64", HIL | SHIFT), (8, 10, 23, 5, "edge", RGEN | INST4),
                                                   (64, 32, 6, 4, "64", HIL | RGEN)])
def test_lobes_fused_step_against_oracle(qmc, d, L, W, H, cname, flags):
    import torch

    from synth import counts_uniform

    P = W * H
    counts = counts_uniform(W, H, 64) if cname == "64" else _counts(P)
    theta = lobe_params(L, d, 6)
    ds, os_ = _pair(qmc, d, 5, flags, W, H)
    ig = qmc.PixelIntegrand.lobes(torch.from_numpy(theta).cuda(), L, d, 9)
    oig = {"kind": "lobes", "d": d, "num_lobes": L, "params": theta, "pixel_seed": 9}
    target = estimator.integrate_pixels(os_, dict(oig, params=perturb(theta, 7)), counts, range(P))["mean"]
    loss64, g64, _ = estimator.loss_and_gradient(os_, oig, counts, range(P), target)
    dc = torch.from_numpy(counts.view(np.int32)).cuda()
    means, loss, grad = qmc.qmc_integrate_pixels_l2_step(ds, ig, W, H, dc,
                                                         torch.from_numpy(target.astype(np.float32)).cuda())
    torch.cuda.synchronize()
    ref = estimator.integrate_pixels(os_, oig, counts, range(P))
    assert _est_tol(means.cpu().numpy(), ref).all()
    g = grad.cpu().numpy().astype(np.float64)
    sizes = estimator.l2_gradient_term_sizes(os_, oig, counts, range(P), target)
    err = np.abs(g - g64)
    ok = (err <= 1e-4 * np.maximum(np.abs(g64), 1e-3 * np.max(np.abs(g64)))) | (err <= 2e-5 * sizes)
    assert ok.all(), (np.nonzero(~ok)[0][:10], g[~ok][:5], g64[~ok][:5], sizes[~ok][:5])
    assert abs(float(loss.cpu()[0]) - loss64) <= 1e-4 * loss64


def test_option_errors(qmc):
    import torch

    W, H = 4, 4
    dc = torch.ones(W * H, dtype=torch.int32, device="cuda")
    ig = qmc.PixelIntegrand.genz(torch.from_numpy(genz_params(W * H, 4)).cuda())
    g = qmc.from_u32(lattice_vector(8, 30, 3))
    with pytest.raises(qmc.QMCError) as e:  # four instances without per-pixel generators
        qmc.qmc_integrate_pixels(qmc.PixelSampler.lattice(g, 1, INST4), ig, W, H, dc)
    assert e.value.status == 1
    from synth import sobol_direction_init
    m = qmc.from_u32(qmc.qmc_sobol_matrices(8, sobol_direction_init(8, 0)))
    with pytest.raises(qmc.QMCError) as e:  # lattice options on the Sobol' sampler
        qmc.qmc_integrate_pixels(qmc.PixelSampler.sobol(m, 1, HIL), ig, W, H, dc)
    assert e.value.status == 1
    big = torch.ones(40000, dtype=torch.int32, device="cuda")
    igb = qmc.PixelIntegrand.genz(torch.zeros((40000, 16), dtype=torch.float32, device="cuda"))
    with pytest.raises(qmc.QMCError) as e:  # Hilbert shift beyond a 32768-pixel side
        qmc.qmc_integrate_pixels(qmc.PixelSampler.lattice(g, 1, HIL), igb, 40000, 1, big)
    assert e.value.status == 2
    torch.cuda.synchronize()
