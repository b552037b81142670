"""Benchmark of the QMC sampling hot path on one MI355X.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-pixels] [--no-progressive]

One step = the scrambled-generation workload: 2^24 points x 32 dims of the Sobol'-type
digital sequence with nested uniform scrambling and an integer Cranley-Patterson rotation,
written as u32 and float32 (4.29 GB), plus the rank-1 lattice sequence n = 2^20, s = 32
with a rotation (268 MB).  Inputs (matrices, seeds, generator vector) are resident on the
GPU before timing starts.  Prints one JSON line.

The same line carries the per-pixel integration workloads ("pixels"): the fused kernels
(generate + evaluate + reduce in one launch, and the adjoint that recomputes samples) timed
next to the plain path (materialise the per-pixel samples in HBM, then integrate them):
  * Genz, 1920x1080 pixels, 2^k samples per pixel (k in 0..8 from a smooth map), d = 8, also
    under the lattice samplers of Sec. 3 and the table-driven samplers of Sec. 2.6.1;
  * Gaussian lobes, 1920x1080 x 64 spp, d = 8, 64 lobes: forward + L2-loss gradient +
    adjoint ("fwd+bwd").
  * the 3840x2160 progressive run: 16 graph-captured passes of 64 spp, d = 64, 32 lobes,
    per-pixel counts in [64, 1024], Sobol' and lattice samplers, and the adjoint over all
    passes (about 10 s; --no-progressive skips it).
"""

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Gpts·dim/s scrambled Sobol'; fused fwd+bwd pixel-samples/s vs plain, %roofline"
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "sobol_scrambled_2p24x32_traffic.json")
KERNEL_SOURCES = ["paper_2307_15584_amd/csrc/generate.hip", "paper_2307_15584_amd/csrc/device_core.hpp"]


def kernel_source_digest():
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(algorithmic_bytes):
    """HBM bytes per launch from the committed counter summary, or None if it is stale."""
    try:
        with open(TRAFFIC_FILE) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_digest") != kernel_source_digest():
        return None
    return rec.get("hbm_bytes_per_launch")


_CPU_SETUP = {}


def _cpu_setup(name):
    """Per-process inputs of the oracle workloads (formed once per worker, outside the timing)."""
    if name in _CPU_SETUP:
        return _CPU_SETUP[name]
    from oracle import digital, estimator
    from synth import (counts_pow2, counts_progressive, counts_uniform, cp_shifts, genz_params, lattice_vector,
                       lobe_params, nus_seeds, sobol_direction_init)

    flags = estimator.PIXEL_NUS | estimator.PIXEL_SHIFT
    if name == "gen":
        v = (digital.sobol_matrices(32, sobol_direction_init(32, 0)), nus_seeds(32, 1), cp_shifts(32, 2),
             lattice_vector(32, 20, 3))
    elif name == "genz":
        m8 = digital.sobol_matrices(8, sobol_direction_init(8, 0))
        v = ({"kind": "sobol", "s": 8, "table": m8, "seed": 0xC3, "flags": flags},
             {"kind": "genz", "d": 8, "pixel_params": genz_params(1920 * 1080, 4)}, counts_pow2(1920, 1080, 5))
    elif name == "lobes":
        m8 = digital.sobol_matrices(8, sobol_direction_init(8, 0))
        v = ({"kind": "sobol", "s": 8, "table": m8, "seed": 0xC3, "flags": flags},
             {"kind": "lobes", "d": 8, "num_lobes": 64, "params": lobe_params(64, 8, 6), "pixel_seed": 9},
             counts_uniform(1920, 1080, 64))
    else:  # progressive 3840x2160, d = 64, 32 lobes
        m64 = digital.sobol_matrices(64, sobol_direction_init(64, 0))
        v = ({"kind": "sobol", "s": 64, "table": m64, "seed": 0xC5, "flags": flags},
             {"kind": "lobes", "d": 64, "num_lobes": 32, "params": lobe_params(32, 64, 6), "pixel_seed": 9},
             counts_progressive(3840, 2160, 5, passes=16, spp_per_pass=64))
    _CPU_SETUP[name] = v
    return v


def _cpu_task(job):
    """One job of an oracle workload; returns (seconds, units of work done)."""
    import numpy as np

    from oracle import estimator, generate

    kind = job[0]
    if kind in ("sobol", "lattice"):
        mats, seeds, shifts, g = _cpu_setup("gen")
        lo, hi = job[1], job[2]
        t0 = time.perf_counter()
        if kind == "sobol":
            generate.generate_sobol(mats, lo, hi - lo, seeds, shifts, 0)
        else:
            generate.generate_lattice(g, lo, hi - lo, shifts, 0)
        return time.perf_counter() - t0, (hi - lo) * 32
    W = 3840 if kind == "progressive" else 1920
    y0, y1, x1 = job[1], job[2], job[3]
    px = (np.arange(y0, y1)[:, None] * W + np.arange(x1)[None, :]).ravel()
    sp, ig, counts = _cpu_setup("genz" if kind == "genz" else "progressive" if kind == "progressive" else "lobes")
    samples = int(counts[px].astype(np.int64).sum())
    t0 = time.perf_counter()
    if kind == "lobes_fwd_bwd":
        estimator.loss_and_gradient(sp, ig, counts, px, np.zeros(len(px)))
    elif kind == "progressive":
        for t in range(16):  # the 16 passes of 64 samples per pixel
            estimator.integrate_pixels(sp, ig, counts, px, begin=64 * t, end=64 * t + 64)
    else:
        estimator.integrate_pixels(sp, ig, counts, px)
    return time.perf_counter() - t0, samples


def _cpu_model():
    """Processor model(s) and the family/model/stepping numbers from /proc/cpuinfo."""
    names, ids = set(), set()
    try:
        with open("/proc/cpuinfo") as fh:
            cur = {}
            for line in fh.read().split("\n") + [""]:
                if not line.strip():
                    if cur:
                        names.add(cur.get("model name", "unknown"))
                        ids.add("family %s model %s stepping %s" % (cur.get("cpu family", "?"), cur.get("model", "?"),
                                                                    cur.get("stepping", "?")))
                    cur = {}
                    continue
                k, _, v = line.partition(":")
                cur[k.strip()] = v.strip()
    except OSError:
        return "unknown"
    return "; ".join(sorted(names)) + " (" + "; ".join(sorted(ids)) + ")"


def cpu_baseline():
    """The oracle (NumPy, exact integers and FP64) on the host cores: the whole generation step
    (scrambled Sobol' 2^24 x 32 and lattice 2^20 x 32) and crops of the pixel workloads, each
    spread over a process pool (all-cores rate) and also reported per core (work / summed job
    time).  The pool has at most 16 processes, the CPU share of one GPU on the benchmark hosts."""
    import multiprocessing as mp

    cores = min(os.cpu_count() or 1, 16)
    ctx = mp.get_context("spawn")
    plans = {
        # name: (jobs, unit, description)
        "sobol": ([("sobol", k << 17, (k + 1) << 17) for k in range(128)], "Gpts·dim/s",
                  "scrambled Sobol' 2^24 x 32 (nested uniform scramble + rotation), u32 + float32"),
        "lattice": ([("lattice", k << 16, (k + 1) << 16) for k in range(16)], "Gpts·dim/s",
                    "rank-1 lattice 2^20 x 32 (rotation), u32 + float32"),
        "genz": ([("genz", 16 * b, 16 * b + 16, 256) for b in range(16)], "pixel-samples/s",
                 "Genz 1920x1080 with 2^k spp: the 256 x 256 top-left crop (its pixels' own seeds and counts)"),
        "lobes_fwd": ([("lobes_fwd", 8 * b, 8 * b + 8, 128) for b in range(16)], "pixel-samples/s",
                      "lobes 1920x1080 x 64 spp, d = 8, 64 lobes, forward: the 128 x 128 top-left crop"),
        "lobes_fwd_bwd": ([("lobes_fwd_bwd", 3 * b, 3 * b + 3, 48) for b in range(16)], "pixel-samples/s",
                          "the same, estimate + L2 loss + analytic gradient: the 48 x 48 top-left crop"),
        "progressive_d64_fwd": ([("progressive", 4 * b, 4 * b + 4, 64) for b in range(16)], "pixel-samples/s",
                                "3840x2160, d = 64, 32 lobes, counts in [64, 1024]: the 64 x 64 top-left crop "
                                "through all 16 passes of 64 spp"),
    }
    out = {}
    with ctx.Pool(cores) as pool:
        pool.map(_cpu_task, [("sobol", 0, 64)] * cores)  # imports, untimed
        for name, (jobs, unit, what) in plans.items():
            kinds = {"sobol": "gen", "lattice": "gen", "genz": "genz", "lobes_fwd": "lobes", "lobes_fwd_bwd": "lobes",
                     "progressive_d64_fwd": "progressive"}
            pool.map(_cpu_setup, [kinds[name]] * (4 * cores), chunksize=1)  # inputs, untimed
            t0 = time.perf_counter()
            res = pool.map(_cpu_task, jobs, chunksize=1)
            wall = time.perf_counter() - t0
            units = sum(r[1] for r in res)
            busy = sum(r[0] for r in res)
            scale = 1e9 if unit == "Gpts·dim/s" else 1.0
            out[name] = {"value": round(units / wall / scale, 4 if scale > 1 else 1), "unit": unit,
                         "value_1core": round(units / busy / scale, 4 if scale > 1 else 1),
                         "work": units, "wall_s": round(wall, 2), "what": what}
    crop = out["progressive_d64_fwd"]
    crop["full_image_seconds_extrapolated"] = round(
        float(_cpu_setup("progressive")[2].astype("int64").sum()) / crop["value"], 1)
    crop["note"] = "full-image time extrapolated from the crop's all-cores rate"
    gen_wall = out["sobol"]["wall_s"] + out["lattice"]["wall_s"]
    ptdims = out["sobol"]["work"] + out["lattice"]["work"]
    return {"value": round(ptdims / gen_wall / 1e9, 4), "unit": "Gpts·dim/s", "cores": cores, "kind": "oracle",
            "sample": "the whole generation step (scrambled Sobol' 2^24 x 32 + lattice 2^20 x 32, u32 + float32) "
                      "in %.1f s on %d processes" % (gen_wall, cores),
            "host_logical_cpus": os.cpu_count(), "cpu": _cpu_model(), "workloads": out}


def _timed(torch, fn, reps, warmup=1):
    """Mean wall ms of fn over reps (synchronised before and after)."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / reps


def _event_ms(torch, fn, reps):
    """Mean GPU ms per call from HIP events around reps back-to-back calls on the current stream."""
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    fn()
    torch.cuda.synchronize()
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    b.synchronize()
    return a.elapsed_time(b) / reps


# ALU roofline of the fused pixel kernels.  One lane-op = one 32-bit VALU operation on one lane;
# the peak is 256 CUs x 2.4 GHz x 2 wave64 instructions per CU per cycle = 78.6 T lane-ops/s.
# Measured (valu_rate probe under counters): adds, multiplies, FMAs and logic sustain about 1.65
# per CU per cycle, multiplies of integers, shifts and conversions 0.94, exp and cos 0.49.
VALU_PEAK_T = 78.6
# index part 1, nested scramble 11, rotation 1, conversion 5 (find-first-bit, shift, and, convert,
# scale by 2^-32); the Genz kernel folds the scale into its integrand constants (4 per dimension)
GEN_OPS_PER_DIM = 18
GENZ_GEN_OPS_PER_DIM = GEN_OPS_PER_DIM - 1
GENZ_EVAL_OPS = 21        # Gaussian 12, phase 4, range reduction 2, exp2 + cos + product 3


def lobe_fwd_ops(d, L):
    """Algorithmic lane-ops per sample of the lobe estimate: generation + offset, then per lobe
    2 per dimension (t = y s + b, E += t^2), exp2 and the weighted sum."""
    return d * (GEN_OPS_PER_DIM + 1) + L * (2 * d + 2)


def lobe_step_ops(d, L):
    """Per sample of the fused estimate + adjoint: per lobe 5 per dimension (t, E, and the three
    adjoint terms) plus exp2, scale, estimate, weight sum and weight product."""
    return d * (GEN_OPS_PER_DIM + 1) + L * (5 * d + 5)


def alu_roofline(samples, ops_per_sample, ms):
    achieved = samples * ops_per_sample / (ms * 1e-3) / 1e12
    return {"bound": "alu", "achieved": round(achieved, 2), "peak": VALU_PEAK_T, "unit": "T lane-ops/s",
            "frac": round(achieved / VALU_PEAK_T, 4), "ops_per_sample": ops_per_sample}


def fill_bandwidth(torch, nbytes=4 << 30, reps=10):
    """Achievable store-only bandwidth (GB/s) of a plain fill of nbytes."""
    buf = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    ms = _timed(torch, lambda: buf.fill_(1.0), reps, 2)
    del buf
    return nbytes / (ms * 1e-3) / 1e9


def pixel_workloads(torch, q, reps, progressive):
    """Fused vs plain per-pixel integration (see the module docstring)."""
    import numpy as np

    from synth import counts_pow2, counts_progressive, counts_uniform, genz_params, lattice_vector, lobe_params
    from synth import nus_seeds, sobol_direction_init, u32_draws

    out = {}
    W, H = 1920, 1080
    P = W * H
    m8 = q.from_u32(q.qmc_sobol_matrices(8, sobol_direction_init(8, 0)))
    sp = q.PixelSampler.sobol(m8, 0xC3)

    # Genz, uneven power-of-two counts
    c3 = counts_pow2(W, H, 5)
    n3 = int(c3.astype(np.int64).sum())
    dc3 = torch.from_numpy(c3.view(np.int32)).cuda()
    ig3 = q.PixelIntegrand.genz(torch.from_numpy(genz_params(P, 4)).cuda())
    q.qmc_autotune_integrate(sp, ig3, W, H, dc3)
    ws3 = torch.empty(max(q.qmc_workspace_size(sp, ig3, W, H), 256), dtype=torch.uint8, device="cuda")
    means = torch.empty(P, dtype=torch.float32, device="cuda")
    fused3 = _timed(torch, lambda: q.qmc_integrate_pixels(sp, ig3, W, H, dc3, means=means, workspace=ws3), reps)
    off3 = q.qmc_sample_offsets(dc3)
    pts3 = torch.empty((8, n3), dtype=torch.float32, device="cuda")
    ptsamp3 = q.PixelSampler.points(pts3, off3)

    def plain3():
        q.qmc_generate_pixel_samples(sp, 8, W, H, dc3, off3, n3, out=pts3)
        q.qmc_integrate_pixels(ptsamp3, ig3, W, H, dc3, means=means, workspace=ws3)

    plain_ms3 = _timed(torch, plain3, reps)
    out["genz_1920x1080_uneven"] = {
        "pixel_samples": n3, "fused_ms": round(fused3, 4), "plain_ms": round(plain_ms3, 4),
        "fused_pixel_samples_per_s": round(n3 / (fused3 * 1e-3), 1),
        "plain_pixel_samples_per_s": round(n3 / (plain_ms3 * 1e-3), 1),
        "speedup_vs_plain": round(plain_ms3 / fused3, 3),
        "roofline": alu_roofline(n3, 8 * GENZ_GEN_OPS_PER_DIM + GENZ_EVAL_OPS, fused3)}
    # the same workload under the lattice samplers of Sec. 3 (shared generator with the pixel's
    # Hilbert shift; per-pixel random generators, four instances)
    gl = q.from_u32(lattice_vector(8, 30, 3))
    lat = {}
    for name, flags in (("pixel_shifted_lattice", q.QMC_PIXEL_HILBERT_SHIFT),
                        ("random_lattice_4_instances", q.QMC_PIXEL_RANDOM_GENERATOR | q.QMC_LATTICE_INSTANCES4
                         | q.QMC_LATTICE_BACKWARD)):
        smp = q.PixelSampler.lattice(gl, 0xC3, flags)
        ms = _timed(torch, lambda: q.qmc_integrate_pixels(smp, ig3, W, H, dc3, means=means, workspace=ws3), reps)
        lat[name] = {"fused_ms": round(ms, 4), "fused_pixel_samples_per_s": round(n3 / (ms * 1e-3), 1)}
    out["genz_1920x1080_uneven"]["lattice_samplers"] = lat
    # and under the table-driven XOR sampler of Sec. 2.6.1: 4096 stored scrambled Sobol' points
    # (made by the library's own generator), 128 x 128 reorder and scramble tables
    stored, _ = q.qmc_generate_sobol(m8, 0, 4096, q.from_u32(nus_seeds(8, 1)), None, want_f32=False)
    xs = q.PixelSampler.xor_table(stored, q.from_u32(u32_draws(21, 8 * q.QMC_XOR_TABLE_CELLS).reshape(8, -1)),
                                  q.from_u32(u32_draws(22, q.QMC_XOR_TABLE_CELLS)))
    ms = _timed(torch, lambda: q.qmc_integrate_pixels(xs, ig3, W, H, dc3, means=means, workspace=ws3), reps)
    out["genz_1920x1080_uneven"]["xor_table_sampler"] = {
        "stored_points": 4096, "fused_ms": round(ms, 4), "fused_pixel_samples_per_s": round(n3 / (ms * 1e-3), 1)}
    # the lattice rotated per pixel from one 128 x 128 table of two-dimensional shifts (Sec. 2.6.1)
    smp = q.PixelSampler.lattice(gl, 0xC3, q.QMC_PIXEL_SHIFT,
                                 shift_table=q.from_u32(u32_draws(23, 2 * q.QMC_XOR_TABLE_CELLS).reshape(2, -1)))
    ms = _timed(torch, lambda: q.qmc_integrate_pixels(smp, ig3, W, H, dc3, means=means, workspace=ws3), reps)
    out["genz_1920x1080_uneven"]["lattice_table_rotations"] = {
        "fused_ms": round(ms, 4), "fused_pixel_samples_per_s": round(n3 / (ms * 1e-3), 1)}
    del pts3

    # Gaussian lobes, forward + L2 gradient + adjoint
    L, d = 64, 8
    c4 = counts_uniform(W, H, 64)
    n4 = P * 64
    dc4 = torch.from_numpy(c4.view(np.int32)).cuda()
    theta = torch.from_numpy(lobe_params(L, d, 6)).cuda()
    ig4 = q.PixelIntegrand.lobes(theta, L, d, 9)
    target = torch.rand(P, device="cuda")
    gm = torch.empty(P, dtype=torch.float32, device="cuda")
    q.qmc_autotune_integrate(sp, ig4, W, H, dc4)
    q.qmc_autotune_integrate(sp, ig4, W, H, dc4, backward=True, grad_means=gm.fill_(1e-7))
    wsf = torch.empty(max(q.qmc_workspace_size(sp, ig4, W, H, False), 256), dtype=torch.uint8, device="cuda")
    wsb = torch.empty(q.qmc_workspace_size(sp, ig4, W, H, True), dtype=torch.uint8, device="cuda")
    grad = torch.zeros(theta.numel(), dtype=torch.float32, device="cuda")

    def fwd_bwd(sampler):
        q.qmc_integrate_pixels(sampler, ig4, W, H, dc4, means=means, workspace=wsf)
        torch.sub(means, target, out=gm).mul_(2.0 / P)
        grad.zero_()
        q.qmc_integrate_pixels_backward(sampler, ig4, W, H, dc4, gm, grad, workspace=wsb)

    wss = torch.empty(q.qmc_workspace_size(sp, ig4, W, H, 2), dtype=torch.uint8, device="cuda")
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")

    def step(sampler):
        loss.zero_()
        grad.zero_()
        q.qmc_integrate_pixels_l2_step(sampler, ig4, W, H, dc4, target, means, loss, grad, workspace=wss)

    fwd_only = _timed(torch, lambda: q.qmc_integrate_pixels(sp, ig4, W, H, dc4, means=means, workspace=wsf), reps)
    two_kernel = _timed(torch, lambda: fwd_bwd(sp), reps)
    fused4 = _timed(torch, lambda: step(sp), reps)
    off4 = q.qmc_sample_offsets(dc4)
    pts4 = torch.empty((d, n4), dtype=torch.float32, device="cuda")
    ptsamp4 = q.PixelSampler.points(pts4, off4)

    def plain4():
        q.qmc_generate_pixel_samples(sp, d, W, H, dc4, off4, n4, out=pts4)
        fwd_bwd(ptsamp4)

    def plain_step():
        q.qmc_generate_pixel_samples(sp, d, W, H, dc4, off4, n4, out=pts4)
        step(ptsamp4)

    plain_ms4 = _timed(torch, plain4, reps)
    plain_step_ms = _timed(torch, plain_step, reps)
    out["lobes_1920x1080x64_fwd_bwd"] = {
        "pixel_samples": n4, "lobes": L, "dims": d, "params": theta.numel(),
        "fused_fwd_ms": round(fwd_only, 4),
        "fused_fwd_bwd_ms": round(fused4, 4),
        "fused_fwd_then_bwd_two_kernels_ms": round(two_kernel, 4),
        "plain_fwd_bwd_ms": round(plain_step_ms, 4),
        "plain_fwd_then_bwd_two_kernels_ms": round(plain_ms4, 4),
        "fused_fwd_bwd_pixel_samples_per_s": round(n4 / (fused4 * 1e-3), 1),
        "plain_fwd_bwd_pixel_samples_per_s": round(n4 / (plain_step_ms * 1e-3), 1),
        "speedup_vs_plain": round(plain_step_ms / fused4, 3),
        "roofline": alu_roofline(n4, lobe_step_ops(d, L), fused4),
        "roofline_fwd": alu_roofline(n4, lobe_fwd_ops(d, L), fwd_only),
        "note": "fused: one kernel samples each pixel once and forms the estimate, the L2 loss gradient and the "
                "adjoint; plain: the samples are materialised in HBM first and the same kernel reads them"}
    del pts4

    if progressive:
        W5, H5, L5, d5 = 3840, 2160, 32, 64
        P5 = W5 * H5
        c5 = counts_progressive(W5, H5, 5, passes=16, spp_per_pass=64)
        n5 = int(c5.astype(np.int64).sum())
        dc5 = torch.from_numpy(c5.view(np.int32)).cuda()
        th5 = torch.from_numpy(lobe_params(L5, d5, 6)).cuda()
        ig5 = q.PixelIntegrand.lobes(th5, L5, d5, 9)
        m64 = q.from_u32(q.qmc_sobol_matrices(64, sobol_direction_init(64, 0)))
        samplers = {"sobol": q.PixelSampler.sobol(m64, 0xC5),
                    "lattice": q.PixelSampler.lattice(q.from_u32(lattice_vector(64, 30, 3)), 0xC5)}
        sums = torch.zeros(P5, dtype=torch.float32, device="cuda")
        means5 = torch.empty(P5, dtype=torch.float32, device="cuda")
        ws5 = torch.empty(max(q.qmc_workspace_size(samplers["sobol"], ig5, W5, H5), 256), dtype=torch.uint8,
                          device="cuda")
        rec = {"pixel_samples": n5, "passes": 16, "spp_per_pass": 64, "dims": d5, "lobes": L5}
        for name, smp in samplers.items():
            def run(graph):
                sums.zero_()
                q.qmc_integrate_progressive(smp, ig5, W5, H5, dc5, 16, 64, sums, means5, ws5, use_graph=graph)
            g_ms = _timed(torch, lambda: run(True), 1)
            e_ms = _timed(torch, lambda: run(False), 1)
            rec[name] = {"graph_ms": round(g_ms, 3), "eager_ms": round(e_ms, 3), "per_pass_ms": round(g_ms / 16, 3),
                         "pixel_samples_per_s": round(n5 / (g_ms * 1e-3), 1),
                         "roofline": alu_roofline(n5, lobe_fwd_ops(d5, L5), g_ms)}
        gm5 = torch.full((P5,), 1e-8, dtype=torch.float32, device="cuda")
        g5 = torch.zeros(th5.numel(), dtype=torch.float32, device="cuda")
        wsb5 = torch.empty(q.qmc_workspace_size(samplers["sobol"], ig5, W5, H5, True), dtype=torch.uint8,
                           device="cuda")
        b_ms = _timed(torch, lambda: q.qmc_integrate_pixels_backward(samplers["sobol"], ig5, W5, H5, dc5, gm5, g5,
                                                                     workspace=wsb5), 1)
        rec["sobol"]["backward_ms"] = round(b_ms, 3)
        rec["sobol"]["backward_roofline"] = alu_roofline(n5, lobe_step_ops(d5, L5), b_ms)
        out["progressive_3840x2160_d64"] = rec
    return out


def pmc_probe(torch, q):
    """A copy of exactly 1 GiB (reads 1 GiB, writes 1 GiB) followed by one scrambled-Sobol'
    generation launch of the benchmark workload, then one launch each of the other 2^24 x 32
    generation kernels (lattice, Halton with identity and Faure digits, partitioned 64-bit
    Sobol' and lattice, point-major Sobol' and lattice), all writing u32 + float32."""
    from synth import cp_shifts, lattice_vector, nus_seeds, sobol_direction_init

    src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    s, n = 32, 1 << 24
    mats = q.from_u32(q.qmc_sobol_matrices(s, sobol_direction_init(s, 0)))
    seeds = q.from_u32(nus_seeds(s, 1))
    shifts = q.from_u32(cp_shifts(s, 2))
    su = torch.empty((s, n), dtype=torch.int32, device="cuda")
    sf = torch.empty((s, n), dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    q.qmc_generate_sobol(mats, 0, n, seeds, shifts, 0, out_u32=su, out_f32=sf)
    torch.cuda.synchronize()
    gvec = q.from_u32(lattice_vector(s, 20, 3))
    wide = q.from_u32(q.qmc_sobol_matrices_wide(s, sobol_direction_init(s, 0), 64))
    others = [
        lambda: q.qmc_generate_lattice(gvec, 0, n, shifts, 0, out_u32=su, out_f32=sf),
        lambda: q.qmc_generate_halton(s, 0, n, q.QMC_HALTON_IDENTITY, None, out_u32=su, out_f32=sf),
        lambda: q.qmc_generate_halton(s, 0, n, q.QMC_HALTON_FAURE, None, out_u32=su, out_f32=sf),
        lambda: q.qmc_generate_sobol64(wide, 1 << 44, n, 8, 77, seeds, shifts, 0, out_u32=su, out_f32=sf),
        lambda: q.qmc_generate_lattice64(gvec, 1 << 44, n, 8, 77, shifts, 0, out_u32=su, out_f32=sf),
        lambda: q.qmc_generate_sobol(mats, 0, n, seeds, shifts, q.QMC_POINT_MAJOR, out_u32=su.view(n, s),
                                     out_f32=sf.view(n, s), ld=s),
        lambda: q.qmc_generate_lattice(gvec, 0, n, shifts, q.QMC_POINT_MAJOR, out_u32=su.view(n, s),
                                       out_f32=sf.view(n, s), ld=s),
    ]
    for fn in others:
        fn()
        torch.cuda.synchronize()
    print("pmc probe done", flush=True)


def pmc_probe_pixels(torch, q):
    """One launch each of the fused pixel kernels on the benchmark workloads, for counter runs:
    Genz forward; lobes d = 8 forward, adjoint and fused L2 step; lobes d = 64 forward and adjoint
    over one 64-spp window of the 3840x2160 image.  The 1920x1080 launch shapes are tuned first,
    as in the benchmark (the tuning launches come first in the counter output; the measured launch
    of each kernel is its last)."""
    import numpy as np

    from synth import counts_pow2, counts_progressive, counts_uniform, genz_params, lobe_params
    from synth import sobol_direction_init

    W, H = 1920, 1080
    P = W * H
    sp = q.PixelSampler.sobol(q.from_u32(q.qmc_sobol_matrices(8, sobol_direction_init(8, 0))), 0xC3)
    dc3 = torch.from_numpy(counts_pow2(W, H, 5).view(np.int32)).cuda()
    ig3 = q.PixelIntegrand.genz(torch.from_numpy(genz_params(P, 4)).cuda())
    dc4 = torch.from_numpy(counts_uniform(W, H, 64).view(np.int32)).cuda()
    ig4 = q.PixelIntegrand.lobes(torch.from_numpy(lobe_params(64, 8, 6)).cuda(), 64, 8, 9)
    gm = torch.full((P,), 1e-7, dtype=torch.float32, device="cuda")
    target = torch.rand(P, device="cuda")
    W5, H5 = 3840, 2160
    dc5 = torch.from_numpy(counts_progressive(W5, H5, 5, passes=16, spp_per_pass=64).view(np.int32)).cuda()
    ig5 = q.PixelIntegrand.lobes(torch.from_numpy(lobe_params(32, 64, 6)).cuda(), 32, 64, 9)
    sp5 = q.PixelSampler.sobol(q.from_u32(q.qmc_sobol_matrices(64, sobol_direction_init(64, 0))), 0xC5)
    gm5 = torch.full((W5 * H5,), 1e-8, dtype=torch.float32, device="cuda")
    q.qmc_autotune_integrate(sp, ig3, W, H, dc3)
    q.qmc_autotune_integrate(sp, ig4, W, H, dc4)
    q.qmc_autotune_integrate(sp, ig4, W, H, dc4, backward=True, grad_means=gm)
    torch.cuda.synchronize()
    for launch in (lambda: q.qmc_integrate_pixels(sp, ig3, W, H, dc3),
                   lambda: q.qmc_integrate_pixels(sp, ig4, W, H, dc4),
                   lambda: q.qmc_integrate_pixels_backward(sp, ig4, W, H, dc4, gm),
                   lambda: q.qmc_integrate_pixels_l2_step(sp, ig4, W, H, dc4, target),
                   lambda: q.qmc_integrate_pixels(sp5, ig5, W5, H5, dc5, 0, 64),
                   lambda: q.qmc_integrate_pixels_backward(sp5, ig5, W5, H5, dc5, gm5, sample_begin=0,
                                                           sample_end=64)):
        launch()
        torch.cuda.synchronize()
    print("pmc pixel probe done", flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline")
    ap.add_argument("--no-pixels", action="store_true", help="skip the per-pixel integration workloads")
    ap.add_argument("--no-progressive", action="store_true", help="skip the 3840x2160 progressive workload")
    ap.add_argument("--progressive", action="store_true", help=argparse.SUPPRESS)  # the default; kept for old commands
    ap.add_argument("--pmc-probe", action="store_true",
                    help="for counter runs: one 1 GiB copy (calibration), then one generation launch; no JSON")
    ap.add_argument("--pmc-probe-pixels", action="store_true",
                    help="for counter runs: one launch each of the fused Genz, lobe forward and lobe adjoint kernels")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path (requested --gpus %d)"
              % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2307_15584_amd as q
    from synth import cp_shifts, lattice_vector, nus_seeds, sobol_direction_init

    torch.cuda.set_device(0)
    if args.pmc_probe:
        pmc_probe(torch, q)
        return
    if args.pmc_probe_pixels:
        pmc_probe_pixels(torch, q)
        return
    fill_gbs = fill_bandwidth(torch)
    s, n = 32, 1 << 24
    nl = 1 << 20
    mats = q.from_u32(q.qmc_sobol_matrices(s, sobol_direction_init(s, 0)))
    seeds = q.from_u32(nus_seeds(s, 1))
    shifts = q.from_u32(cp_shifts(s, 2))
    gvec = q.from_u32(lattice_vector(s, 20, 3))
    su = torch.empty((s, n), dtype=torch.int32, device="cuda")
    sf = torch.empty((s, n), dtype=torch.float32, device="cuda")
    lu = torch.empty((s, nl), dtype=torch.int32, device="cuda")
    lf = torch.empty((s, nl), dtype=torch.float32, device="cuda")

    def step(ev=None):
        if ev is not None:
            ev[0].record()
        q.qmc_generate_sobol(mats, 0, n, seeds, shifts, 0, out_u32=su, out_f32=sf)
        if ev is not None:
            ev[1].record()
        q.qmc_generate_lattice(gvec, 0, nl, shifts, 0, out_u32=lu, out_f32=lf)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    events = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(events[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    sobol_ms = float(np.mean([a.elapsed_time(b) for a, b in events]))

    ms_per_step = wall * 1e3 / args.steps
    ptdims = s * n + s * nl
    value = ptdims / (ms_per_step * 1e-3) / 1e9
    alg_bytes = s * n * 8
    achieved = alg_bytes / (sobol_ms * 1e-3) / 1e9
    traffic = measured_traffic(alg_bytes)
    out = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "Gpts·dim/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "scrambled Sobol' 2^24 x 32 dims (nested uniform scramble + integer rotation, "
                               "u32 + float32 out) + rank-1 lattice 2^20 x 32 dims (rotation, u32 + float32 out)",
                   "points_sobol": n, "points_lattice": nl, "dims": s, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "kernel": "sobol_fast (scramble + rotation, u32 + f32)",
                     "kernel_ms": round(sobol_ms, 4), "algorithmic_bytes": alg_bytes,
                     "fill_gbs": round(fill_gbs, 1), "frac_of_fill": round(achieved / fill_gbs, 4)},
    }
    # the other generation workloads: lattice at the Sobol' size (steady-state roofline) and the
    # small unscrambled (0,2)-sequence + 2 dims (launch latency)
    q.qmc_generate_lattice(gvec, 0, n, shifts, 0, out_u32=su, out_f32=sf)
    lat_ms = _event_ms(torch, lambda: q.qmc_generate_lattice(gvec, 0, n, shifts, 0, out_u32=su, out_f32=sf), 20)
    out["lattice_2p24x32"] = {"kernel_ms": round(lat_ms, 4), "gbs": round(alg_bytes / (lat_ms * 1e-3) / 1e9, 1),
                              "frac": round(alg_bytes / (lat_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    # the same scrambled Sobol' workload written as u32 only (2.15 GB)
    u32_ms = _event_ms(torch, lambda: q.qmc_generate_sobol(mats, 0, n, seeds, shifts, 0, out_u32=su, want_f32=False),
                       10)
    out["sobol_u32_only_2p24x32"] = {"kernel_ms": round(u32_ms, 4),
                                     "gpts_dim_per_s": round(s * n / (u32_ms * 1e-3) / 1e9, 1),
                                     "hbm_frac": round(alg_bytes / 2 / (u32_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    hal = {}
    for name, mode in (("identity", q.QMC_HALTON_IDENTITY), ("faure", q.QMC_HALTON_FAURE)):
        h_ms = _event_ms(torch, lambda: q.qmc_generate_halton(s, 0, n, mode, None, out_u32=su, out_f32=sf), 10)
        hal[name] = {"kernel_ms": round(h_ms, 4), "gpts_dim_per_s": round(s * n / (h_ms * 1e-3) / 1e9, 1),
                     "hbm_frac": round(alg_bytes / (h_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    out["halton_2p24x32"] = hal
    pm_u = su.view(n, s)
    pm_f = sf.view(n, s)
    pm_ms = _event_ms(torch, lambda: q.qmc_generate_sobol(mats, 0, n, seeds, shifts, q.QMC_POINT_MAJOR, out_u32=pm_u,
                                                          out_f32=pm_f, ld=s), 5)
    out["sobol_point_major_2p24x32"] = {"kernel_ms": round(pm_ms, 4),
                                        "gpts_dim_per_s": round(s * n / (pm_ms * 1e-3) / 1e9, 1),
                                        "hbm_frac": round(alg_bytes / (pm_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    lpm_ms = _event_ms(torch, lambda: q.qmc_generate_lattice(gvec, 0, n, shifts, q.QMC_POINT_MAJOR, out_u32=pm_u,
                                                              out_f32=pm_f, ld=s), 5)
    out["lattice_point_major_2p24x32"] = {"kernel_ms": round(lpm_ms, 4),
                                          "gpts_dim_per_s": round(s * n / (lpm_ms * 1e-3) / 1e9, 1),
                                          "hbm_frac": round(alg_bytes / (lpm_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    # 64-bit indices and partitioned enumeration: part 77 of 2^8 from m = 2^44 (global indices
    # near 2^52), the same 2^24 x 32 scrambled + rotated workload as the headline kernel
    wide = q.from_u32(q.qmc_sobol_matrices_wide(s, sobol_direction_init(s, 0), 64))
    w_ms = _event_ms(torch, lambda: q.qmc_generate_sobol64(wide, 1 << 44, n, 8, 77, seeds, shifts, 0, out_u32=su,
                                                            out_f32=sf), 10)
    l64_ms = _event_ms(torch, lambda: q.qmc_generate_lattice64(gvec, 1 << 44, n, 8, 77, shifts, 0, out_u32=su,
                                                                out_f32=sf), 10)
    out["partitioned_64bit_2p24x32"] = {
        "sobol_kernel_ms": round(w_ms, 4), "sobol_hbm_frac": round(alg_bytes / (w_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "lattice_kernel_ms": round(l64_ms, 4),
        "lattice_hbm_frac": round(alg_bytes / (l64_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "note": "part 77 of 2^8, subsequence indices from 2^44; cost of 64-bit indices = ratio to the 32-bit kernels"}
    m4 = q.from_u32(q.qmc_sobol_matrices(4, sobol_direction_init(4, 0)))
    c1u = torch.empty((4, 1 << 16), dtype=torch.int32, device="cuda")
    c1f = torch.empty((4, 1 << 16), dtype=torch.float32, device="cuda")
    c1_ms = _event_ms(torch, lambda: q.qmc_generate_sobol(m4, 0, 1 << 16, None, None, 0, out_u32=c1u, out_f32=c1f),
                      200)
    out["unscrambled_2p16x4"] = {"us_per_launch": round(c1_ms * 1e3, 2),
                                 "note": "kernel time from HIP events around 200 back-to-back launches"}
    del su, sf, lu, lf, c1u, c1f
    torch.cuda.empty_cache()
    if not args.no_pixels:
        out["pixels"] = pixel_workloads(torch, q, max(3, args.steps // 4), not args.no_progressive)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
