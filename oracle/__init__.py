"""CPU oracle for the QMC sampling and integration path — TEST INFRASTRUCTURE ONLY.

A plain, slow, obviously correct implementation of what the GPU library computes,
written from Keller, Waechter and Binder, "Quasi-Monte Carlo Algorithms (not only)
for Graphics Software" (arXiv 2307.15584).  Integers are exact (numpy uint64 with
explicit 32-bit masks, or Python ints) and floating point is FP64 unless the paper
fixes the precision.

Only the test suite, the smoke check and the CPU-baseline leg of the benchmark may
import this package.  It shares no code with the HIP library and imports nothing
from it; the only common dependency is `synth`, which draws seeded inputs.

Modules:
  unifloat    map_u32_to_unifloat (Sec. 2.1, Alg. 1)
  digital     radical inverse phi_2, primitive polynomials, Sobol' generator
              matrices and points (Sec. 2.2, 2.3, Eq. ts)
  scramble    nested uniform scramble, shifts, the per-pixel hash (Sec. 2.1, 2.3, 2.5.2)
  lattice     rank-1 lattice sequence points (Sec. 2.4, Eq. R1LS, Alg. 4)
  pixel_lattice  per-pixel lattices of Sec. 3: random generator per pixel (Alg. 4),
              radical inverse in base b, Hilbert index, pixel-shifted lattice
              (Eq. PixelShiftedR1LS)
  halton      radical inversion in prime bases with identity, Faure or linear digit
              permutations, and the Halton sequence (Sec. 2.2)
  partition   64-bit indices (wide Sobol' matrices, 64-digit lattice) and the partitioned
              enumeration of one sequence across processing elements (Sec. 2.5.1)
  xor_table   the table-driven per-pixel samplers of Sec. 2.6.1: stored points with a
              per-pixel index reordering and digit scramble by XOR, and per-pixel rotations
              from one 128 x 128 table of two-dimensional shifts
  integrands  Genz and Gaussian-lobe integrands and their parameter gradients
  estimator   per-pixel QMC integro-approximation, loss, analytic and
              finite-difference gradients (Sec. 2.5)

Parity status: the nested uniform scramble is builder-defined (the paper cites Owen
scrambling without fixing one); its arithmetic has no external value to pin against,
so its *values* are "parity unpinned" and only its defining properties are pinned
(nestedness, bijectivity, net preservation).  The per-pixel hash and the integrands
are likewise builder-defined workloads, pinned by their published definition
(hash) and by closed-form integrals and finite differences (integrands).  The per-pixel
random lattice generator (a hash the paper leaves open) is "parity unpinned" in the
same way: only its oddness and distinctness are pinned.
"""
