"""Benchmark of the QMC sampling hot path on one MI355X.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--extra]

One step = the scrambled-generation workload: 2^24 points x 32 dims of the Sobol'-type
digital sequence with nested uniform scrambling and an integer Cranley-Patterson rotation,
written as u32 and float32 (4.29 GB), plus the rank-1 lattice sequence n = 2^20, s = 32
with a rotation (268 MB).  Inputs (matrices, seeds, generator vector) are resident on the
GPU before timing starts.  Prints one JSON line.
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


def _cpu_job(args):
    lo, hi = args
    import numpy as np  # noqa: F401

    from oracle import digital, generate
    from synth import cp_shifts, nus_seeds, sobol_direction_init

    s = 32
    mats = digital.sobol_matrices(s, sobol_direction_init(s, 0))
    t0 = time.perf_counter()
    generate.generate_sobol(mats, lo, hi - lo, nus_seeds(s, 1), cp_shifts(s, 2), 0)
    return time.perf_counter() - t0


def cpu_baseline(points=1 << 21, chunks=64):
    """The oracle on a bounded sample of the same workload (first `points` indices, 32 dims)."""
    import multiprocessing as mp

    cores = min(os.cpu_count() or 1, 16)
    step = points // chunks
    jobs = [(k * step, (k + 1) * step) for k in range(chunks)]
    ctx = mp.get_context("spawn")
    with ctx.Pool(cores) as pool:
        pool.map(_cpu_job, [(0, 64)] * cores)  # import warm-up, untimed
        t0 = time.perf_counter()
        pool.map(_cpu_job, jobs)
        wall = time.perf_counter() - t0
    ptdims = points * 32
    return {"value": ptdims / wall / 1e9, "unit": "Gpts·dim/s", "cores": cores, "kind": "oracle",
            "sample": "first %d indices x 32 dims, scramble + rotation, u32 + float32; %.1f s wall on %d "
                      "processes" % (points, wall, cores)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline")
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
                     "kernel_ms": round(sobol_ms, 4), "algorithmic_bytes": alg_bytes},
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
