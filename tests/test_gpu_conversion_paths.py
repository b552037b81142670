"""The float conversion of Sec. 2.1 as the per-pixel kernels compute it, over all 2^32 inputs.

The materialising generators convert with the hardware's round-toward-zero conversion; the
per-pixel kernels, whose other FP32 arithmetic rounds to nearest, normalise with a leading-zero
count and scale by a power of two instead.  This test drives that second form through the C ABI:
the table-driven XOR sampler (Sec. 2.6.1) of a 128 x 128 image, one dimension, every pixel 2^13
samples, stored points k = 0 .. 2^27 - 1, reorder entry c 2^13 for cell c (so sample i of pixel
p reads stored point p 2^13 + i) and every digit scramble equal to the top five bits of the
chunk.  The materialised samples are then the conversions of 2^27 consecutive integers, compared
bit for bit with the oracle, chunk by chunk (as the paper checked its conversion, Sec. 2.1).
"""

import os

import numpy as np
import pytest

from _exhaustive import compare_slice

pytestmark = pytest.mark.gpu

CELLS = 16384


def test_pixel_kernel_conversion_exhaustive(qmc):
    import multiprocessing as mp
    from multiprocessing import shared_memory

    import torch

    W = H = 128
    P = W * H
    spp = 1 << 13
    chunk = P * spp  # 2^27
    counts = torch.full((P,), spp, dtype=torch.int32, device="cuda")
    offs = qmc.qmc_sample_offsets(counts)
    stored = torch.arange(chunk, dtype=torch.int32, device="cuda").view(1, chunk)
    reorder = (torch.arange(CELLS, dtype=torch.int64, device="cuda") << 13).to(torch.int32)
    out = torch.empty((1, chunk), dtype=torch.float32, device="cuda")
    workers = min(16, os.cpu_count() or 1)
    ctx = mp.get_context("spawn")
    shm = shared_memory.SharedMemory(create=True, size=chunk * 4)
    host = np.ndarray((chunk,), dtype=np.uint32, buffer=shm.buf)
    try:
        with ctx.Pool(workers) as pool:
            for c in range(32):
                start = c << 27
                top = start - (1 << 32) if start >= (1 << 31) else start
                scramble = torch.full((1, CELLS), top, dtype=torch.int32, device="cuda")
                sampler = qmc.PixelSampler.xor_table(stored, scramble, reorder)
                qmc.qmc_generate_pixel_samples(sampler, 1, W, H, counts, offs, chunk, out=out)
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
