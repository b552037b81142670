"""The fused lobe kernels' in-register samples are the library's materialised samples, bit for
bit (A22 reading: the fused kernels do not store their scrambled points, so their bit-exactness
is shown through their results).

The materialised per-pixel samples are checked bit for bit against the oracle elsewhere.  Here
the same kernels run twice: once generating their samples in registers (scrambled Sobol' or
rotated lattice), once reading the materialised samples (the POINTS sampler).  Both walks visit
the samples in the same order and evaluate the same arithmetic, so any difference in a single
sample bit would show as a different result.  Covered: the forward estimate, the adjoint and
the fused L2 step at d = 8 (one lobe group and two), d = 64 (two lanes per sample, each forming
32 dimensions) and d = 40 (the second half partly empty), with empty, packed and big pixels.
"""

import numpy as np
import pytest

from synth import counts_uniform, lattice_vector, lobe_params, sobol_direction_init

pytestmark = pytest.mark.gpu

NUS, SHIFT, BACK = 4, 8, 2


def _counts_edge(P):
    base = np.array([0, 1, 2, 3, 63, 64, 65, 127, 128, 129, 200, 256, 5, 31, 32, 33, 1000], dtype=np.uint32)
    return np.resize(base, P)


CASES = [
    # d, L, W, H, counts, sampler kind, flags
    (8, 64, 37, 5, "edge", "sobol", NUS | SHIFT),
    (8, 100, 16, 4, "64", "sobol", NUS | SHIFT),      # two lobe groups
    (64, 32, 9, 4, "edge", "sobol", NUS | SHIFT),     # two lanes per sample
    (64, 32, 8, 4, "64", "lattice", SHIFT | BACK),
    (40, 33, 7, 5, "edge", "sobol", NUS | SHIFT),     # second half of the dimensions partly unused
]


def _u32(t):
    return t.detach().cpu().numpy().view(np.uint32)


@pytest.mark.parametrize("case", CASES, ids=["d%d-L%d-%s-%s" % (c[0], c[1], c[4], c[5]) for c in CASES])
def test_plain_equals_fused_lobe_kernels_bitwise(qmc, case):
    import torch

    d, L, W, H, cname, kind, flags = case
    P = W * H
    counts = counts_uniform(W, H, 64) if cname == "64" else _counts_edge(P)
    s = max(d, 8)
    if kind == "sobol":
        table = qmc.from_u32(qmc.qmc_sobol_matrices(s, sobol_direction_init(s, 0)))
        fused = qmc.PixelSampler.sobol(table, 0x5EED, flags)
    else:
        fused = qmc.PixelSampler.lattice(qmc.from_u32(lattice_vector(s, 30, 3)), 0x5EED, flags)
    dc = torch.from_numpy(counts.view(np.int32)).cuda()
    offs = qmc.qmc_sample_offsets(dc)
    total = int(counts.astype(np.int64).sum())
    pts = qmc.qmc_generate_pixel_samples(fused, d, W, H, dc, offs, total)
    plain = qmc.PixelSampler.points(pts, offs)
    theta = torch.from_numpy(lobe_params(L, d, 6)).cuda()
    ig = qmc.PixelIntegrand.lobes(theta, L, d, 11)
    gm = torch.from_numpy(np.random.default_rng(12).uniform(-1, 1, P).astype(np.float32) / P).cuda()
    target = torch.from_numpy(np.random.default_rng(13).uniform(0, 1, P).astype(np.float32)).cuda()

    res = {}
    for name, smp in (("fused", fused), ("plain", plain)):
        means = qmc.qmc_integrate_pixels(smp, ig, W, H, dc)
        grad = qmc.qmc_integrate_pixels_backward(smp, ig, W, H, dc, gm)
        sm, sl, sg = qmc.qmc_integrate_pixels_l2_step(smp, ig, W, H, dc, target)
        torch.cuda.synchronize()
        res[name] = [_u32(t) for t in (means, grad, sm, sl, sg)]
    for k, what in enumerate(("forward means", "adjoint", "L2-step means", "L2-step loss", "L2-step gradient")):
        a, b = res["fused"][k], res["plain"][k]
        assert np.array_equal(a, b), (what, np.nonzero(a != b)[0][:10])
