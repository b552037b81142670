"""Seeded synthetic inputs shared by the CPU oracle, the tests and the benchmark.

This package only draws random numbers and lays them out; it holds none of the
sampling or integration arithmetic.  Every stream is SplitMix64 (Steele, Lea and
Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014) keyed by an
explicit integer seed, so the inputs are identical on every machine and numpy
version.
"""

from .inputs import (  # noqa: F401
    MAX_DEGREE,
    splitmix64,
    uniform01,
    u32_draws,
    sobol_direction_init,
    nus_seeds,
    cp_shifts,
    lattice_vector,
    genz_params,
    value_noise,
    counts_pow2,
    counts_progressive,
    counts_uniform,
    lobe_params,
    perturb,
    pick,
)
