"""Worker for the exhaustive float-conversion check: compares a slice of GPU results held
in shared memory with the oracle (runs in spawned processes, imports no GPU code)."""

import numpy as np


def compare_slice(args):
    shm_name, total, start_u, lo, hi = args
    from multiprocessing import shared_memory

    from oracle.unifloat import map_u32_to_unifloat_bits

    shm = shared_memory.SharedMemory(name=shm_name)
    try:
        got = np.ndarray((total,), dtype=np.uint32, buffer=shm.buf)[lo:hi]
        u = np.arange(start_u + lo, start_u + hi, dtype=np.uint64)
        want = map_u32_to_unifloat_bits(u)
        bad = np.nonzero(got != want)[0]
        first_bad = int(start_u + lo + bad[0]) if bad.size else -1
        return int(bad.size), first_bad
    finally:
        shm.close()
