"""The C ABI allocates nothing and copies nothing between host and device per call, so every
call can be captured in a HIP graph.  A graph holding the generation calls (Sobol', lattice,
Halton, partitioned 64-bit Sobol') and the fused L2 step is replayed several times, with eager
work between the replays, and every replay must reproduce the eager results bit for bit."""

import numpy as np
import pytest

from oracle import digital, partition
from synth import counts_uniform, cp_shifts, lattice_vector, lobe_params, nus_seeds, sobol_direction_init

pytestmark = pytest.mark.gpu


def test_generation_and_l2_step_replay_in_a_graph(qmc):
    import torch

    s, n = 8, 3 * 4096 + 100
    dev = "cuda"
    mats = qmc.from_u32(digital.sobol_matrices(s, sobol_direction_init(s, 0)))
    wide = qmc.from_u32(partition.sobol_matrices_wide(s, sobol_direction_init(s, 0), 64))
    seeds, shifts = qmc.from_u32(nus_seeds(s, 1)), qmc.from_u32(cp_shifts(s, 2))
    gvec = qmc.from_u32(lattice_vector(s, 20, 3))
    outs_u = [torch.empty((s, n), dtype=torch.int32, device=dev) for _ in range(4)]
    outs_f = [torch.empty((s, n), dtype=torch.float32, device=dev) for _ in range(4)]

    W, H, L, d = 24, 16, 64, 8
    P = W * H
    dc = torch.from_numpy(counts_uniform(W, H, 64).view(np.int32)).to(dev)
    theta = lobe_params(L, d, 6)
    ig = qmc.PixelIntegrand.lobes(torch.from_numpy(theta).to(dev), L, d, 9)
    sp = qmc.PixelSampler.sobol(mats, 0xC4)
    target = torch.from_numpy(np.random.default_rng(7).random(P).astype(np.float32)).to(dev)
    means = torch.empty(P, dtype=torch.float32, device=dev)
    loss = torch.zeros(1, dtype=torch.float32, device=dev)
    grad = torch.zeros(theta.size, dtype=torch.float32, device=dev)
    ws = torch.empty(qmc.qmc_workspace_size(sp, ig, W, H, 2), dtype=torch.uint8, device=dev)

    def work():
        qmc.qmc_generate_sobol(mats, 0, n, seeds, shifts, 0, out_u32=outs_u[0], out_f32=outs_f[0])
        qmc.qmc_generate_lattice(gvec, 4, n, shifts, 0, out_u32=outs_u[1], out_f32=outs_f[1])
        qmc.qmc_generate_halton(s, 8, n, qmc.QMC_HALTON_FAURE, None, out_u32=outs_u[2], out_f32=outs_f[2])
        qmc.qmc_generate_sobol64(wide, 1 << 40, n, 3, 5, seeds, shifts, 0, out_u32=outs_u[3], out_f32=outs_f[3])
        loss.zero_()
        grad.zero_()
        qmc.qmc_integrate_pixels_l2_step(sp, ig, W, H, dc, target, means, loss, grad, workspace=ws)

    results = outs_u + outs_f + [means, loss, grad]
    work()
    torch.cuda.synchronize()
    ref = [t.clone() for t in results]

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        work()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        work()
    torch.cuda.synchronize()
    for rep in range(3):
        for t in results:
            t.fill_(-7)                     # eager work between replays
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for k, (t, r) in enumerate(zip(results, ref)):
            assert torch.equal(t, r), (rep, k)
    # the step's estimates agree with the forward kernel's (a different kernel: FP32 rounding)
    fresh = qmc.qmc_integrate_pixels(sp, ig, W, H, dc)
    torch.cuda.synchronize()
    assert torch.allclose(fresh, ref[-3], rtol=2e-5, atol=0)
