"""The allocation-free training step (static per-device scratch) against the step that takes a
workspace: same kernels, so the means, loss and gradient agree bit for bit.  Two calls in a row,
the second on a smaller problem, so that what the first left in the shared scratch cannot leak
into the second; and a problem beyond the scratch's limit is refused before any launch."""

import numpy as np
import pytest

from synth import lobe_params, sobol_direction_init

pytestmark = pytest.mark.gpu

NUS, SHIFT = 4, 8


def _counts(P):
    base = np.array([0, 1, 2, 3, 63, 64, 65, 127, 128, 129, 200, 256, 5, 31, 32, 33, 1000], dtype=np.uint32)
    return np.resize(base, P)


def _problem(qmc, d, L, W, H, seed):
    import torch

    P = W * H
    s = max(d, 8)
    mats = qmc.from_u32(qmc.qmc_sobol_matrices(s, sobol_direction_init(s, 0)))
    sp = qmc.PixelSampler.sobol(mats, seed, NUS | SHIFT)
    theta = torch.from_numpy(lobe_params(L, d, 6)).cuda()
    ig = qmc.PixelIntegrand.lobes(theta, L, d, 9)
    dc = torch.from_numpy(_counts(P).view(np.int32)).cuda()
    target = torch.from_numpy(np.random.default_rng(seed).uniform(0, 1, P).astype(np.float32)).cuda()
    return sp, ig, dc, target, theta.numel()


def _u32(t):
    return t.detach().cpu().numpy().view(np.uint32)


def test_noalloc_step_equals_workspace_step_twice(qmc):
    import torch

    for d, L, W, H, seed in ((64, 32, 20, 13, 5), (8, 16, 9, 5, 6)):
        sp, ig, dc, target, n = _problem(qmc, d, L, W, H, seed)
        P = W * H
        ref = qmc.qmc_integrate_pixels_l2_step(sp, ig, W, H, dc, target)
        means = torch.empty(P, dtype=torch.float32, device="cuda")
        loss = torch.zeros(1, dtype=torch.float32, device="cuda")
        grad = torch.zeros(n, dtype=torch.float32, device="cuda")
        got = qmc.qmc_integrate_pixels_l2_step_noalloc(sp, ig, W, H, dc, target, means, loss, grad)
        torch.cuda.synchronize()
        for what, a, b in zip(("means", "loss", "gradient"), ref, got):
            assert np.array_equal(_u32(a), _u32(b)), (d, L, what)
        assert np.isfinite(_u32(grad).view(np.float32)).all() and float(loss[0]) > 0.0


def test_noalloc_step_refuses_problems_beyond_the_scratch(qmc):
    import torch

    W, H, L, d = 8, 8, 400, 8   # 400 x 17 = 6800 parameters > 6550
    sp, ig, dc, target, n = _problem(qmc, d, L, W, H, 7)
    assert qmc.qmc_workspace_size(sp, ig, W, H, 2) > qmc.QMC_STATIC_SCRATCH_BYTES
    means = torch.empty(W * H, dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    grad = torch.zeros(n, dtype=torch.float32, device="cuda")
    with pytest.raises(qmc.QMCError) as e:
        qmc.qmc_integrate_pixels_l2_step_noalloc(sp, ig, W, H, dc, target, means, loss, grad)
    assert e.value.status == 5 and "static scratch" in str(e.value)
    # the largest lobe count that fits at d = 8: 385 lobes (6545 parameters <= 6550)
    sp, ig, dc, target, n = _problem(qmc, 8, 385, W, H, 8)
    assert qmc.qmc_workspace_size(sp, ig, W, H, 2) <= qmc.QMC_STATIC_SCRATCH_BYTES
    ref = qmc.qmc_integrate_pixels_l2_step(sp, ig, W, H, dc, target)
    grad = torch.zeros(n, dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    got = qmc.qmc_integrate_pixels_l2_step_noalloc(sp, ig, W, H, dc, target, means, loss, grad)
    torch.cuda.synchronize()
    for a, b in zip(ref, got):
        assert np.array_equal(_u32(a), _u32(b))
