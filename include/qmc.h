/*
 * qmc.h -- C ABI of the MI355X (gfx950) quasi-Monte Carlo sampling library.
 *
 * Implements the data-parallel core of Keller, Waechter and Binder, "Quasi-Monte Carlo
 * Algorithms (not only) for Graphics Software" (arXiv 2307.15584): digital sequences
 * (Sec. 2.3, Eq. ts), rank-1 lattice sequences (Sec. 2.4, Eq. R1LS), randomisation kept
 * in integers (Sec. 2.1, 2.3, 2.5.2) and the float conversion map_u32_to_unifloat
 * (Sec. 2.1, Alg. 1), batched over indices and dimensions, and fused into per-pixel
 * QMC integro-approximation (Sec. 2.5) with an adjoint for parameter gradients.
 *
 * Conventions for every call:
 *   - Pointers marked "device" are HIP device allocations owned by the caller; the
 *     library never frees, retains or allocates them, and performs no host<->device copy.
 *     Pointers marked "host" are ordinary host memory, read or written before return.
 *   - Work is enqueued on `stream` (a hipStream_t; NULL = the null stream of the current
 *     device) and is asynchronous: results are visible after the stream is synchronised.
 *     No call synchronises the stream, so every call may be captured in a hipGraph.
 *   - Arguments are validated on the host before anything is enqueued; a non-OK status
 *     means nothing was enqueued.  qmc_last_error() then describes the problem.  A fault
 *     inside a kernel surfaces at the caller's next synchronisation, as a HIP error.
 *   - Index ranges are 32-bit: first + n <= 2^32 is required (Sec. 2.5 warns that a
 *     silently wrapping index is hard to find, so a range that would wrap is rejected).
 *   - Integer samples are u32 fixed-point fractions: value v stands for v * 2^-32.
 */
#ifndef QMC_H
#define QMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    QMC_OK = 0,
    QMC_ERR_INVALID_ARGUMENT = 1, /* null pointer, zero dimension count, bad flags, ld < n, ... */
    QMC_ERR_OUT_OF_RANGE = 2,     /* index range beyond 2^32, too many dimensions, ...         */
    QMC_ERR_UNSUPPORTED = 3,      /* a valid request this build does not implement              */
    QMC_ERR_DEVICE = 4,           /* a HIP runtime call failed                                  */
    QMC_ERR_WORKSPACE = 5         /* caller-provided workspace too small                        */
} qmc_status;

/* Opaque per-device state: device properties, tuned launch parameters and captured
 * graphs.  It holds no caller buffers.  One context may be used from one thread at a time. */
typedef struct qmc_context_s* qmc_context;

/* A hipStream_t, passed as an untyped handle so that this header needs no HIP headers. */
typedef void* qmc_stream;

#define QMC_MAX_DIMS 64   /* dimensions per call (s) */
#define QMC_MAX_DEGREE 16 /* initial direction numbers per dimension */

/* flags */
#define QMC_SHIFT_XOR 1u        /* shift by XOR (digital shift, Sec. 2.3) instead of addition mod 2^32 */
#define QMC_LATTICE_BACKWARD 2u /* lattice: enumerate phi_2(2^32-1-i) so the origin comes last (Alg. 4) */
#define QMC_POINT_MAJOR 128u    /* generation: out[(i-first)*ld + j] (ld >= s) instead of out[j*ld + (i-first)] */

/* ---------------------------------------------------------------- context ---- */

/* Create a context for HIP device `device`.  *out receives the handle.
 * Errors: INVALID_ARGUMENT (out NULL), DEVICE (no such device / HIP failure). */
qmc_status qmc_create(int device, qmc_context* out);

/* Destroy a context and everything it owns (tuned parameters, graphs).  NULL is a no-op. */
qmc_status qmc_destroy(qmc_context ctx);

/* Text of the last non-OK status returned on the calling thread ("" if none).  The string
 * is owned by the library and valid until the next call on this thread. */
const char* qmc_last_error(void);

/* Library version string, e.g. "qmc-gfx950 1.0". */
const char* qmc_version(void);

/* ------------------------------------------------------------------ setup ---- */

/* The first `count` primitive polynomials over F_2, ordered by degree and then by their
 * integer code (bit t = coefficient of x^t), written to host array codes[count].
 * They define Sobol' dimensions 1.. (Sec. 2.3).  Errors: INVALID_ARGUMENT (codes NULL),
 * OUT_OF_RANGE (count > 4096). */
qmc_status qmc_primitive_polynomials(uint32_t count, uint32_t* codes);

/* Sobol' generator matrices for s dimensions (Sec. 2.3, Eq. ts), written to host array
 * matrices[s][32]: column k (= matrices[j*32+k]) is the image of index bit k, and bit 31
 * of a column is the coefficient of 2^-1.  Dimension 0 is the identity (van der Corput);
 * dimension j >= 1 uses the (j-1)-th primitive polynomial of degree d with initial
 * direction numbers direction_init[j*QMC_MAX_DEGREE + 0 .. d-1] (host; odd, m_k < 2^k)
 * and the Sobol' recurrence for the rest.
 * Errors: INVALID_ARGUMENT (NULL, an even or too large m_k), OUT_OF_RANGE (s > QMC_MAX_DIMS
 * or s == 0, or a polynomial degree above QMC_MAX_DEGREE). */
qmc_status qmc_sobol_matrices(uint32_t s, const uint32_t* direction_init, uint32_t* matrices);

/* The same matrices for indices of up to `columns` bits (the 64-bit index form of Alg. 3),
 * written to host array matrices[s][columns]: column k (= matrices[j*columns+k]) keeps the top
 * 32 digits of the fraction m_(k+1) 2^-(k+1), i.e. m_(k+1) << (31-k) for k < 32 and
 * m_(k+1) >> (k-31) for k >= 32; dimension 0 has zero columns from 32 on.  The first 32
 * columns equal qmc_sobol_matrices'.  columns: 1..64.  Errors as for qmc_sobol_matrices,
 * plus OUT_OF_RANGE for columns outside [1, 64]. */
qmc_status qmc_sobol_matrices_wide(uint32_t s, const uint32_t* direction_init, uint32_t columns,
                                   uint32_t* matrices);

/* ------------------------------------------------------------- generation ---- */

/* Halton sequence (Sec. 2.2): component j of point i is
 *   v = floor(2^32 phi_{b_j,sigma}(i mod b_j^M)),   x = map_u32_to_unifloat(v),
 * with b_j the j-th prime (2, 3, 5, ..., 311 for j < 64), b_j^M the largest power of b_j that
 * fits in 32 bits (the listing's max_powers), and phi_{b,sigma}(k) = sum_t sigma(a_t(k)) b^(-t-1)
 * for the base-b digits a_t(k).  The digit permutation sigma is chosen by `mode`:
 *   QMC_HALTON_IDENTITY  sigma(a) = a;
 *   QMC_HALTON_FAURE     Faure's permutations (Sec. 2.2): sigma_2 = (0,1); even b: 2 sigma_{b/2}
 *                        followed by 2 sigma_{b/2} + 1; odd b: sigma_{b-1} with values
 *                        >= (b-1)/2 raised by one and (b-1)/2 inserted in the middle;
 *   QMC_HALTON_LINEAR    sigma(a) = (factors[j] * a) mod b_j (linear digit scrambling; the
 *                        paper's multiplier table is not printed, so the caller supplies it;
 *                        a factor that is 0 mod b_j maps every digit to 0; not checked).
 * Output (dimension-major), first/n/ld rules, alignment fast path and errors as for
 * qmc_generate_sobol without flags.
 *   s:        1..QMC_MAX_DIMS.
 *   factors:  device u32 [s], required for QMC_HALTON_LINEAR, else ignored (may be NULL). */
#define QMC_HALTON_IDENTITY 0u
#define QMC_HALTON_FAURE 1u
#define QMC_HALTON_LINEAR 2u
qmc_status qmc_generate_halton(qmc_context ctx, qmc_stream stream, uint32_t s, uint64_t first, uint64_t n,
                               uint32_t mode, const uint32_t* factors, uint32_t* out_u32, float* out_f32,
                               uint64_t ld);

/* map_u32_to_unifloat (Sec. 2.1, Alg. 1) over an array: out[k] = the largest binary32 not
 * above in[k] * 2^-32, so every result lies in [0, 1).  in, out: device, n elements each
 * (may alias exactly).  Errors: INVALID_ARGUMENT (NULL with n > 0). */
qmc_status qmc_map_u32_to_unifloat(qmc_context ctx, qmc_stream stream,
                                   const uint32_t* in, float* out, uint64_t n);

/* Points i in [first, first+n) of an s-dimensional digital sequence in base 2 (Eq. ts),
 * randomised in integers and converted (Sec. 2.1):
 *     v = C_j a(i)                       generator-matrix product over F_2
 *     v = NUS(v; nus_seeds[j])           if nus_seeds != NULL (nested uniform scramble)
 *     v = v + shifts[j] mod 2^32         if shifts != NULL (v ^ shifts[j] with QMC_SHIFT_XOR)
 *     out_u32[j*ld + (i-first)] = v,  out_f32[j*ld + (i-first)] = map_u32_to_unifloat(v)
 * NUS(x; s) = brev(P_s(brev(x))) where brev mirrors the 32 bits and P_s is, mod 2^32 with
 * lo24(v) = v & 0xFFFFFF:  v += s;  v += lo24(v)*0x612362;  v ^= v<<8;
 * v += lo24(v)*((s>>8)&0xFFFFFE);  v += lo24(v)*0x934C76;  v ^= v<<9;  v ^= v*0xFA8F38AA.
 * Each output digit is the input digit flipped by a function of the seed and of the more
 * significant digits only (a nested uniform scramble in the sense of Owen, cited in
 * Sec. 2.1 and 2.5.2), so digital-net properties are preserved.
 *   matrices:  device, [s][32] u32 as produced by qmc_sobol_matrices (any matrices allowed).
 *   nus_seeds, shifts: device [s] u32, or NULL.
 *   out_u32, out_f32: device, dimension-major with leading dimension ld >= n; either may be
 *              NULL but not both.  Outputs must not overlap each other or the inputs.
 *   flags:     0, QMC_SHIFT_XOR, QMC_POINT_MAJOR (point-major layout: out[(i-first)*ld + j] with
 *              ld >= s; then an output spans ((n-1)*ld + s) words).
 * Errors: INVALID_ARGUMENT (NULL inputs, both outputs NULL, ld < n, unknown flags),
 *         OUT_OF_RANGE (s == 0 or s > QMC_MAX_DIMS, first + n > 2^32). n == 0 is a no-op. */
qmc_status qmc_generate_sobol(qmc_context ctx, qmc_stream stream,
                              const uint32_t* matrices, uint32_t s,
                              uint64_t first, uint64_t n,
                              const uint32_t* nus_seeds, const uint32_t* shifts,
                              uint32_t flags,
                              uint32_t* out_u32, float* out_f32, uint64_t ld);

/* Points i in [first, first+n) of the rank-1 lattice sequence (Sec. 2.4, Eq. R1LS) in
 * base 2 with generator vector g (Alg. 4):
 *     v = phi_2(i) * g_j mod 1, computed as brev(i) * g_j mod 2^32
 *         (brev(2^32-1-i) * g_j with QMC_LATTICE_BACKWARD, so the origin comes last)
 *     v = v + shifts[j] mod 2^32 if shifts != NULL (v ^ shifts[j] with QMC_SHIFT_XOR)
 *     outputs as for qmc_generate_sobol.
 *   generator: device [s] u32 (odd components give a Latin hypercube at 2^m points).
 * Errors as for qmc_generate_sobol; flags may combine QMC_SHIFT_XOR, QMC_LATTICE_BACKWARD and
 * QMC_POINT_MAJOR. */
qmc_status qmc_generate_lattice(qmc_context ctx, qmc_stream stream,
                                const uint32_t* generator, uint32_t s,
                                uint64_t first, uint64_t n,
                                const uint32_t* shifts, uint32_t flags,
                                uint32_t* out_u32, float* out_f32, uint64_t ld);

/* 64-bit indices and partitioned enumeration (Sec. 2.5.1; the 64-bit index of Alg. 3).
 * One sequence is split among 2^log2_parts processing elements by an extra splitting
 * dimension, the van der Corput sequence phi_2(i): part p receives, in index order, the
 * indices whose phi_2 lies in [p 2^-q, (p+1) 2^-q) (q = log2_parts), which are exactly
 *     i(m) = m 2^q + rev_q(p),   m = 0, 1, 2, ...      (rev_q mirrors the q low bits)
 * These calls write points m in [first, first+n) of part p, dimension-major as
 * qmc_generate_sobol: out[j*ld + (m-first)].  q = 0 (one part, p = 0) gives the sequence
 * itself with 64-bit indices i = m.
 *
 * Digital sequence: v = C_j a(i) over all `columns` index bits with matrices [s][columns]
 * from qmc_sobol_matrices_wide (any matrices allowed); then NUS, shift and conversion exactly
 * as qmc_generate_sobol.  Every index must be below 2^columns:
 *     first + n <= 2^(columns - q), else OUT_OF_RANGE (no index bit is dropped silently).
 *   columns:    1..64;  log2_parts: 0..min(32, columns);  part < 2^log2_parts.
 *   flags:      0 or QMC_SHIFT_XOR (QMC_POINT_MAJOR is not available here).
 * Errors: as qmc_generate_sobol, with OUT_OF_RANGE for columns, log2_parts, part and the
 * index range above.  n may exceed 2^32 (the output then spans more than 16 GiB). */
qmc_status qmc_generate_sobol64(qmc_context ctx, qmc_stream stream,
                                const uint32_t* matrices, uint32_t columns, uint32_t s,
                                uint32_t log2_parts, uint32_t part,
                                uint64_t first, uint64_t n,
                                const uint32_t* nus_seeds, const uint32_t* shifts,
                                uint32_t flags,
                                uint32_t* out_u32, float* out_f32, uint64_t ld);

/* Rank-1 lattice sequence with 64-bit indices (Eq. R1LS over all 64 binary digits):
 *     v = floor(2^32 frac(phi_2(i) g_j)) = ((brev64(i) g_j) mod 2^64) >> 32
 * (phi_2(2^64-1-i) with QMC_LATTICE_BACKWARD), then shift and conversion as
 * qmc_generate_lattice, over the indices i(m) of part p above.  For i < 2^32 the value equals
 * qmc_generate_lattice's forward one.  Index range: first + n <= 2^(64 - q).
 *   flags: QMC_SHIFT_XOR, QMC_LATTICE_BACKWARD.
 * Errors: as qmc_generate_sobol64. */
qmc_status qmc_generate_lattice64(qmc_context ctx, qmc_stream stream,
                                  const uint32_t* generator, uint32_t s,
                                  uint32_t log2_parts, uint32_t part,
                                  uint64_t first, uint64_t n,
                                  const uint32_t* shifts, uint32_t flags,
                                  uint32_t* out_u32, float* out_f32, uint64_t ld);

/* ------------------------------------------------- per-pixel integration ---- */
/*
 * Integro-approximation over an image (Sec. 2.5, Sec. 3): pixel p = y * width + x
 * (row-major) estimates I_p = (1/N_p) sum_{i < N_p} f_p(x_{p,i}) with N_p = counts[p]
 * samples.  Every pixel owns an independently randomised copy of the sequence (Sec.
 * 2.5.2), so pixels need no communication and their sample counts may differ.  A call
 * covers the sample window i in [sample_begin, min(sample_end, N_p)) of every pixel, so
 * a run can be split into progressive passes whose sums add up exactly.
 *
 * Sample i of pixel p, dimension j < d (integers until the last step, Sec. 2.1):
 *   SOBOL:   v = C_j a(i);  v = NUS(v; seed_pj) with QMC_PIXEL_NUS;
 *   LATTICE: v = (phi_2(i) + s_p) g_j mod 1 (phi_2(2^32-1-i) with QMC_LATTICE_BACKWARD), in
 *            32-bit fixed point; s_p = 0 unless QMC_PIXEL_HILBERT_SHIFT (below); g_j = table[j]
 *            unless QMC_PIXEL_RANDOM_GENERATOR (below);
 *   then v = v + delta_pj mod 2^32 with QMC_PIXEL_SHIFT (v ^ delta_pj with QMC_SHIFT_XOR),
 *   and x = map_u32_to_unifloat(v).
 *   seed_pj  = H(H(seed + 2j) ^ p),  delta_pj = H(H(seed + 2j + 1) ^ p), where H is the
 *   integer hash "pcg" of Jarzynski and Olano (JCGT 2020):
 *   t = v*747796405 + 2891336453; w = ((t >> ((t >> 28) + 4)) ^ t) * 277803737; H = (w >> 22) ^ w.
 *   QMC_PIXEL_TABLE_SHIFT (with QMC_PIXEL_SHIFT; Sec. 2.6.1, one table of two-dimensional
 *     rotations repeated for all pairs of dimensions): delta_pj = shift_table[(j mod 2) *
 *     16384 + c] for the pixel's cell c = (y mod 128) * 128 + (x mod 128), instead of the hash.
 * Lattice options of Sec. 3:
 *   QMC_PIXEL_RANDOM_GENERATOR (Alg. 4): pixel p's own generator, g_pj = H(H(H(seed + 2j) ^ p)
 *     + c) | 1 for instance c = 0 (the table is still read but its values are not used);
 *   QMC_LATTICE_INSTANCES4 (with the above): four instances superimposed in each pixel, sample
 *     i being point floor(i / 4) of instance c = i mod 4;
 *   QMC_PIXEL_HILBERT_SHIFT (Eq. PixelShiftedR1LS): s_p = floor(2^32 phi_3(h(x, y))), h the
 *     index of pixel (x, y) along the Hilbert curve of the 2^k x 2^k square, 2^k the smallest
 *     power of two >= max(width, height) (at most 32768), visiting the quadrants of every
 *     square in the order (0,0), (0,1), (1,1), (1,0) (x = column, y = row) with the
 *     sub-curves of the two quadrants at y < half transposed (the one at x >= half about the
 *     other diagonal), so that consecutive indices are edge-adjacent pixels.
 *   POINTS:  x = table[j * points_ld + offsets[p] + i] (samples materialised beforehand by
 *   qmc_generate_pixel_samples: the plain generate-then-integrate path).
 *   XOR_TABLE (Sec. 2.6.1, image-plane decorrelation by XOR): one set of N stored integer
 *     points P_j[k] = table[j * points_ld + k], N = points_ld a power of two, serves every
 *     pixel; for the pixel's cell c = (y mod 128) * 128 + (x mod 128) of the 128 x 128 tables,
 *     v = P_j[(i XOR xor_reorder[c]) mod N] XOR xor_scramble[j * 16384 + c], then
 *     x = map_u32_to_unifloat(v).  The stored points (Owen-scrambled Sobol' points in the
 *     paper, e.g. from qmc_generate_sobol with NUS) and both tables are the caller's; the
 *     index is taken modulo N, so the stored points repeat with period N.  No flags.
 *
 * Integrands (FP32 on the GPU):
 *   QMC_F_GENZ (d = 8; pixel_params [P][16]: centres u_0..u_7 then widths a_0..a_7):
 *     f_p(x) = exp(-sum_{j<4} a_j^2 (x_j - u_j)^2) * cos(2 pi u_4 + sum_{j=4..7} a_j x_j)
 *   QMC_F_LOBES (shared theta = [centres c (L x d), log-widths l (L x d), weights w (L)]):
 *     f_p(x) = sum_k w_k exp(-1/2 sum_j ((x_j + delta'_pj - c_kj) e^{-l_kj})^2), with the
 *     per-pixel offset delta'_pj = fl(fl(0.5 * map_u32_to_unifloat(H(H(pixel_seed + j) ^ p)))
 *     - 0.25) in [-1/4, 1/4) and x_j + delta'_pj rounded to binary32.
 */
#define QMC_SAMPLER_SOBOL 1u
#define QMC_SAMPLER_LATTICE 2u
#define QMC_SAMPLER_POINTS 3u
#define QMC_SAMPLER_XOR_TABLE 4u
#define QMC_XOR_TABLE_CELLS 16384u      /* 128 x 128 cells of the XOR_TABLE sampler's tables */

#define QMC_PIXEL_NUS 4u                /* sampler flag: per-pixel nested uniform scramble (SOBOL) */
#define QMC_PIXEL_SHIFT 8u              /* sampler flag: per-pixel rotation (addition, or XOR with QMC_SHIFT_XOR) */
#define QMC_PIXEL_RANDOM_GENERATOR 16u  /* LATTICE: per-pixel random generator vector (Alg. 4) */
#define QMC_PIXEL_HILBERT_SHIFT 32u     /* LATTICE: Hilbert-curve shift of phi_2 (Eq. PixelShiftedR1LS) */
#define QMC_LATTICE_INSTANCES4 64u      /* LATTICE with QMC_PIXEL_RANDOM_GENERATOR: four instances */
#define QMC_PIXEL_TABLE_SHIFT 256u      /* SOBOL/LATTICE with QMC_PIXEL_SHIFT: rotations from shift_table */

#define QMC_F_GENZ 1u
#define QMC_F_LOBES 2u

typedef struct {
    uint32_t kind;           /* QMC_SAMPLER_*                                                     */
    uint32_t s;              /* dimensions in `table` (>= the integrand's d; <= QMC_MAX_DIMS)      */
    const void* table;       /* device: SOBOL u32 [s][32] matrices | LATTICE u32 [s] generator |   */
                             /*         POINTS float32 [s][points_ld] samples |                    */
                             /*         XOR_TABLE u32 [s][points_ld] stored points                 */
    uint64_t points_ld;      /* POINTS: leading dimension of table; XOR_TABLE: N, a power of two  */
                             /*         in [1, 2^32]                                               */
    const uint64_t* offsets; /* POINTS: device [P], slot of sample 0 of pixel p                    */
    uint32_t seed;           /* per-pixel seeds and rotations are derived from this                */
    uint32_t flags;          /* QMC_PIXEL_NUS | QMC_PIXEL_SHIFT | QMC_SHIFT_XOR | QMC_LATTICE_BACKWARD  */
                             /* | QMC_PIXEL_RANDOM_GENERATOR | QMC_LATTICE_INSTANCES4                  */
                             /* | QMC_PIXEL_HILBERT_SHIFT (the last three: LATTICE only)              */
                             /* | QMC_PIXEL_TABLE_SHIFT (with QMC_PIXEL_SHIFT)                        */
    const uint32_t* xor_scramble; /* XOR_TABLE: device u32 [s][16384] digit scrambles s_cj         */
    const uint32_t* xor_reorder;  /* XOR_TABLE: device u32 [16384] index reorderings r_c           */
    const uint32_t* shift_table;  /* QMC_PIXEL_TABLE_SHIFT: device u32 [2][16384] rotation vectors  */
} qmc_sampler;

typedef struct {
    uint32_t kind;             /* QMC_F_GENZ or QMC_F_LOBES                                      */
    uint32_t d;                /* dimensions consumed: 8 for GENZ; 1..QMC_MAX_DIMS for LOBES     */
    uint32_t num_lobes;        /* LOBES: L >= 1                                                  */
    uint32_t pixel_seed;       /* LOBES: seed of the per-pixel offsets                           */
    const float* params;       /* LOBES: device theta [L*(2d+1)]                                 */
    const float* pixel_params; /* GENZ: device [P][16]                                           */
} qmc_integrand;

/* Bytes of device workspace needed by qmc_integrate_pixels (backward = 0), by
 * qmc_integrate_pixels_backward (backward = 1) or by qmc_integrate_pixels_l2_step
 * (backward = 2) for this problem, in *bytes.  The workspace holds 1024 bytes of task counters
 * and, for the adjoint, an exact accumulator of 640 bytes per gradient entry (n_theta entries,
 * plus the loss for the L2 step): 1024 + 640 * n_row bytes, bounded by the parameter count and
 * not by the image size (2.6 MB for 4128 parameters); for the GENZ forward pass, the list of
 * the P pixels sorted into buckets by sample count and the buckets' counts per 1024 pixels:
 * about 4 P + 360 ceil(P / 1024) + 6144 bytes (9.0 MB at 1920 x 1080).
 * Errors: INVALID_ARGUMENT (NULL), UNSUPPORTED (kind/dimension combination). */
qmc_status qmc_workspace_size(qmc_context ctx, const qmc_sampler* sampler, const qmc_integrand* integrand,
                              uint32_t width, uint32_t height, int backward, size_t* bytes);

/* Adds the window sums to sums[p] (if sums != NULL) and writes means[p] = sums[p] / N_p
 * (or window sum / N_p if sums is NULL; 0 where N_p = 0) if means != NULL.  One persistent
 * launch covers all pixels whatever their counts; per-pixel sums are reduced in a fixed
 * order, so results are bitwise reproducible for a given launch configuration.
 *   counts: device u32 [width*height];  sums, means: device float32 [width*height];
 *   workspace: device, >= qmc_workspace_size(..., 0) bytes, no initial contents required.
 * Errors: INVALID_ARGUMENT (NULLs, sums and means both NULL, d > s, bad flags, begin > end,
 *         XOR_TABLE without its tables or with N not a power of two in [1, 2^32],
 *         QMC_PIXEL_TABLE_SHIFT without QMC_PIXEL_SHIFT or without shift_table),
 *         UNSUPPORTED (d not supported for the kind), WORKSPACE (too small). */
qmc_status qmc_integrate_pixels(qmc_context ctx, qmc_stream stream, const qmc_sampler* sampler,
                                const qmc_integrand* integrand, uint32_t width, uint32_t height,
                                const uint32_t* counts, uint32_t sample_begin, uint32_t sample_end,
                                float* sums, float* means, void* workspace, size_t workspace_bytes);

/* Adjoint of qmc_integrate_pixels for QMC_F_LOBES: given grad_means[p] = dL/dI_p, adds
 *   dL/dtheta = sum_p grad_means[p] / N_p * sum_{i in window} df_p(x_{p,i}) / dtheta
 * to grad_params[L*(2d+1)] (device float32; the caller zeroes it for a fresh gradient).
 * Samples are recomputed from (p, i) rather than stored.  Each tile of 64 pixels forms its
 * float32 partial gradient; the partials are summed exactly (as integer multiples of 2^-149 in
 * 64-bit words) and the exact sum is rounded once, so the result is bitwise reproducible and the
 * same for every launch configuration and schedule.
 * workspace: >= qmc_workspace_size(..., 1) bytes.
 * Errors as for qmc_integrate_pixels; UNSUPPORTED for integrands other than LOBES. */
qmc_status qmc_integrate_pixels_backward(qmc_context ctx, qmc_stream stream, const qmc_sampler* sampler,
                                         const qmc_integrand* integrand, uint32_t width, uint32_t height,
                                         const uint32_t* counts, uint32_t sample_begin, uint32_t sample_end,
                                         const float* grad_means, float* grad_params, void* workspace,
                                         size_t workspace_bytes);

/* One fused training step for the per-pixel L2 loss L = (1/P) sum_p (I_p - T_p)^2 of the
 * lobe integrand over the full windows [0, N_p): estimates I_p, dL/dI_p = 2 (I_p - T_p) / P
 * and the adjoint of qmc_integrate_pixels_backward, in one launch (plus the rounding of the
 * exact sums of the gradient and of the loss).  The adjoint's per-pixel sums do not depend on dL/dI_p, only their scaling
 * does, so with at most 64 lobes (32 when d > 32) one pass over each pixel's samples
 * accumulates the estimate and the unscaled adjoint sums together and scales them when the
 * pixel is complete: samples are generated once.  With more lobes the forward pass over all
 * lobes precedes the adjoint pass (samples are generated again).
 *   target: device float32 [P];  means: device float32 [P] or NULL (written);
 *   loss: device float32 [1], L is added;  grad_params: device float32 [L*(2d+1)], added.
 *   workspace: >= qmc_workspace_size(..., 2) bytes.
 * Errors as for qmc_integrate_pixels_backward. */
qmc_status qmc_integrate_pixels_l2_step(qmc_context ctx, qmc_stream stream, const qmc_sampler* sampler,
                                        const qmc_integrand* integrand, uint32_t width, uint32_t height,
                                        const uint32_t* counts, const float* target, float* means, float* loss,
                                        float* grad_params, void* workspace, size_t workspace_bytes);

/* For callers that cannot allocate device memory: code under HIP graph capture, tight serving or
 * training loops, harnesses that forbid allocation.  The same step as
 * qmc_integrate_pixels_l2_step (same kernels, bitwise the same results) without a workspace
 * argument: its work counter and exact accumulator live in the library's static scratch of
 * QMC_STATIC_SCRATCH_BYTES per device (held by every device the library runs on until the
 * process ends).  The call allocates nothing and launches kernels only.  Limit: the problem's
 * qmc_workspace_size(..., 2), 1024 + 640 (L (2d+1) + 1) bytes, must not exceed
 * QMC_STATIC_SCRATCH_BYTES, i.e. L (2d+1) <= 6550 parameters; larger problems fail with
 * WORKSPACE before anything is enqueued.  Every call on one device shares that device's scratch
 * and clears what it needs at its start, so calls that overlap on one GPU (other streams, other
 * threads, other contexts of the device) race and must be ordered by the caller.
 * Arguments, outputs and the other errors as for qmc_integrate_pixels_l2_step. */
#define QMC_STATIC_SCRATCH_BYTES (4u << 20)
qmc_status qmc_integrate_pixels_l2_step_noalloc(qmc_context ctx, qmc_stream stream, const qmc_sampler* sampler,
                                                const qmc_integrand* integrand, uint32_t width, uint32_t height,
                                                const uint32_t* counts, const float* target, float* means,
                                                float* loss, float* grad_params);

/* Exclusive prefix sums of counts: offsets[p] = sum_{q<p} counts[q] (device u64 [num_pixels+1],
 * offsets[num_pixels] = total).  workspace: >= 8 * (num_pixels / 1024 + 2) bytes.  Used to lay
 * out materialised per-pixel samples. */
qmc_status qmc_sample_offsets(qmc_context ctx, qmc_stream stream, const uint32_t* counts, uint32_t num_pixels,
                              uint64_t* offsets, void* workspace, size_t workspace_bytes);

/* The plain path's first half: writes sample i < N_p of pixel p, dimension j < d, as
 * out[j * ld + offsets[p] + i] (float32), exactly the values the fused integration uses
 * (before any integrand offset).  sampler: SOBOL, LATTICE or XOR_TABLE.  offsets: from
 * qmc_sample_offsets; ld >= offsets[P]; out: device float32 [d][ld].
 * workspace: >= 1024 bytes of device memory (work counters). */
qmc_status qmc_generate_pixel_samples(qmc_context ctx, qmc_stream stream, const qmc_sampler* sampler, uint32_t d,
                                      uint32_t width, uint32_t height, const uint32_t* counts,
                                      const uint64_t* offsets, float* out, uint64_t ld, void* workspace,
                                      size_t workspace_bytes);

/* ------------------------------------------- progressive passes (graphs) ---- */

/* Progressive integration (Sec. 2.5: every pixel extends its own sequence, so passes are
 * added without communication): pass t covers the sample window [t*spp_per_pass,
 * (t+1)*spp_per_pass) of every pixel (pixels with N_p below the window contribute nothing),
 * adding into sums; the last pass also writes means (if not NULL).  With use_graph != 0 the
 * passes are captured once into a hipGraph (on a private stream of the context), cached in
 * the context under all arguments, and replayed on `stream` with hipGraphLaunch; otherwise
 * they are enqueued one by one.  The sums after all passes equal one call with the window
 * [0, passes*spp_per_pass) up to FP32 summation order.
 *   sums: device float32 [P], required; workspace as for qmc_integrate_pixels.
 * Errors: as for qmc_integrate_pixels; OUT_OF_RANGE if passes*spp_per_pass >= 2^32;
 *         DEVICE if capture or instantiation fails. */
qmc_status qmc_integrate_progressive(qmc_context ctx, qmc_stream stream, const qmc_sampler* sampler,
                                     const qmc_integrand* integrand, uint32_t width, uint32_t height,
                                     const uint32_t* counts, uint32_t passes, uint32_t spp_per_pass, float* sums,
                                     float* means, void* workspace, size_t workspace_bytes, int use_graph);

/* ------------------------------------------------------------- autotuning ---- */

/* Times each launch shape of the materialising kernels (1, 2, 4 or 8 chunks of 256 indices per
 * wavefront, with and without non-temporal stores) on `stream` with hipEvents and keeps the fastest in the context
 * for that sequence kind.  The candidates write the n points of `table` into the caller's
 * scratch buffers ([s][n] each; either may be NULL but not both).  Synchronises `stream`
 * (not capturable).  report (may be NULL) receives one JSON line per candidate.
 * kind: QMC_SAMPLER_SOBOL (table = matrices, nus_seeds/shifts optional) or
 * QMC_SAMPLER_LATTICE (table = generator, shifts optional). */
qmc_status qmc_autotune_generate(qmc_context ctx, qmc_stream stream, uint32_t kind, const uint32_t* table,
                                 uint32_t s, uint64_t n, const uint32_t* nus_seeds, const uint32_t* shifts,
                                 uint32_t* scratch_u32, float* scratch_f32, char* report, size_t report_bytes);

/* Times the integration launch shapes (persistent grid of 4..32 wavefronts per compute unit,
 * static or atomic-queue schedule) for this problem and keeps the fastest in the context for
 * (integrand kind, d, direction); among shapes within 1 % of the fastest, the one with the
 * fewest wavefronts per compute unit.  Forward candidates write means into scratch (device
 * float32 [P]); backward candidates (backward != 0, grad_means required) add gradients into
 * scratch (device float32 [n_theta]).  Synchronises `stream`.  report as above. */
qmc_status qmc_autotune_integrate(qmc_context ctx, qmc_stream stream, const qmc_sampler* sampler,
                                  const qmc_integrand* integrand, uint32_t width, uint32_t height,
                                  const uint32_t* counts, uint32_t sample_begin, uint32_t sample_end, int backward,
                                  const float* grad_means, float* scratch, void* workspace, size_t workspace_bytes,
                                  char* report, size_t report_bytes);

/* Write / read the context's tuned launch parameters as JSON (host file path). */
qmc_status qmc_tune_save(qmc_context ctx, const char* path);
qmc_status qmc_tune_load(qmc_context ctx, const char* path);

#ifdef __cplusplus
}
#endif

#endif /* QMC_H */
