// Per-pixel QMC integro-approximation (Sec. 2.5): every pixel integrates with its own
// randomised copy of a low-discrepancy sequence (Sec. 2.5.2), so pixels are independent and
// only a final per-pixel reduction is needed; counts may differ from pixel to pixel.
//
// Work decomposition (one persistent launch, any mix of counts):
//   * a task is a tile of kTile = 64 consecutive pixels; wavefronts take tasks from a
//     static interleave or from an atomic queue (chosen per problem by the autotuner);
//   * lane q of the wavefront reads the count of pixel q of the tile;
//   * pixels with at least 64 samples in the window ("big") are processed one at a time by
//     the whole wavefront: their per-dimension seeds are computed by lanes j < d once and
//     shared through LDS, and lane l takes samples l, l+64, ...;
//   * the remaining pixels are packed: their samples are laid end to end and processed 64
//     per round, one per lane;
//   * sample index i = begin + k of dimension j is C_j (begin + k); with begin a multiple of
//     64 it splits into a per-round part (advanced by one XOR per round, like the
//     materialising kernels) and a per-lane part C_j k, k < 64, from an LDS table.
// Consumers of the samples:
//   * Genz (per-pixel parameters): one sample per lane; big pixels accumulate per lane and
//     finish with one butterfly reduction, packed pixels with a segmented scan per round;
//   * Gaussian lobes (parameters shared by all pixels), forward and adjoint: each round of
//     samples is staged in LDS and every lane owns one lobe (for d > 32, half of a lobe's
//     dimensions, so 32 lobes still fill a wavefront): t_j = fma(y_j, st_j, b_j) with
//     st = sqrt(log2(e)/2) e^-l and b = -c st, E = sum t_j^2, G = exp2(-E).  The forward pass
//     reduces across lanes once per pixel; the adjoint needs no cross-lane reduction at all:
//     at the end of a task each lane adds its lobe's partial gradient into an exact accumulator.
// Exact accumulation: a float32 value is m 2^(e-150) with an integer m < 2^24, so it is an
// integer multiple of 2^-149 below 2^128.  Each value is split into two 32-bit digits of that
// integer (position fixed by its exponent) and the digits are added with 64-bit integer atomics
// into nine int64 words per parameter (32-bit digit positions with 32 bits of headroom for
// carries).  Integer addition is associative, so the sum is exact and the same whichever
// wavefront added which task in which order; one final kernel propagates the carries and rounds
// once to float.  Several copies of the words (by block) spread the atomics.
// Results never depend on which wavefront ran which task, so they are bitwise reproducible.
#include <cmath>
#include <mutex>

#include "common.hpp"
#include "device_core.hpp"

namespace qmc {

IntegrateTune& integrate_tune(qmc_context ctx, uint32_t fkind, uint32_t d, bool backward);

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x4_a4 __attribute__((ext_vector_type(4), aligned(4)));  // four floats at any 4-byte boundary
typedef uint32_t u32x4_a4 __attribute__((ext_vector_type(4), aligned(4)));

constexpr uint32_t kWave = 64;
constexpr uint32_t kTile = 64;   // pixels per task
constexpr uint32_t kQI = 26;     // stride entries for index bits 6..31
constexpr uint32_t kBlock = 256;
constexpr uint32_t kWavesPerBlock = kBlock / kWave;
constexpr float kKappa = 0.84932180028801904f;  // sqrt(log2(e) / 2): exp(-r^2/2) = exp2(-(kKappa r)^2)
// Exact accumulator (see the top of file): digit words per parameter (nine for the digit
// positions of finite floats, one counting non-finite values) and copies of the words.
constexpr uint32_t kAccDigits = 9;
constexpr uint32_t kAccWords = 10;
constexpr uint32_t kAccCopies = 8;

struct Args {
    // sampler
    uint32_t skind, s, seed, sflags;
    uint32_t sxor;  // shift by XOR instead of addition
    // lattice options of Sec. 3: per-pixel random generator (Alg. 4), four superimposed
    // instances, Hilbert-curve shift of the radical inverse (Eq. PixelShiftedR1LS)
    uint32_t lrgen, linst4, lhilbert;
    uint32_t width, hilbert_order;  // image width; 2^hilbert_order >= max(width, height)
    const uint32_t* table;
    const float* points;
    uint64_t points_ld;
    const uint64_t* offsets;
    // table-driven XOR sampler (Sec. 2.6.1): digit scrambles [s][cells], index reorderings
    // [cells], and N - 1 for the N stored points in `table`
    const uint32_t* xor_scramble;
    const uint32_t* xor_reorder;
    uint32_t xor_mask;
    // rotations from a 128 x 128 table of two-dimensional shifts [2][cells] (Sec. 2.6.1), or NULL
    const uint32_t* shift_table;
    // integrand
    uint32_t fkind, d, L, pixel_seed;
    const float* params;        // theta (lobes)
    const float* pixel_params;  // Genz [P][16]
    // problem
    uint32_t num_pixels;
    const uint32_t* counts;
    uint32_t begin, end;
    uint32_t aligned;  // begin % 64 == 0
    float* sums;
    float* means;
    const float* grad_means;
    const float* target;  // L2 step: per-pixel targets
    // materialised samples (plain path)
    float* out;
    uint64_t out_ld;
    // schedule
    uint32_t num_tasks;
    uint32_t* queue;
    uint32_t dynamic;
    uint32_t total_waves;
    // Genz buckets (see genz_bucket_count): sizes [kBuckets], per-wavefront counts
    // [kBuckets][bucket_waves], pixel list [P]
    uint32_t* bucket_total;
    uint32_t* bucket_wave;
    uint32_t* bucket_list;
    uint32_t bucket_waves;
    // Genz, Sobol' sampler: index-part tables (see genz_tables), read through the scalar cache
    uint32_t* genz_tab;
    // adjoint: exact accumulators [kAccCopies][n_row][kAccWords], n_row = n_theta (+1 for the
    // loss sum of the L2 step)
    unsigned long long* acc;
    uint32_t n_theta, n_row;
};

// -------------------------------------------------------------- wave helpers ----

__device__ __forceinline__ uint32_t lane_id() { return threadIdx.x & (kWave - 1); }

// Orders this wavefront's LDS writes before its later LDS reads by other lanes.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

// The same sum in DPP, without LDS: an inclusive scan (row shifts by 1, 2, 4, 8, then row
// broadcasts of lanes 15 and 31) leaves the total in lane 63, which is returned to every lane.
// Used where it measured faster: at the end of each big pixel of the Genz kernel (the lobe
// kernels measured the same or slower with it).
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_add(float v) {
    return v + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROW_MASK, 0xF, false));
}

__device__ __forceinline__ float wave_sum_dpp(float v) {
    v = dpp_add<0x111, 0xF>(v);
    v = dpp_add<0x112, 0xF>(v);
    v = dpp_add<0x114, 0xF>(v);
    v = dpp_add<0x118, 0xF>(v);
    v = dpp_add<0x142, 0xA>(v);
    v = dpp_add<0x143, 0xC>(v);
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

__device__ __forceinline__ uint32_t wave_excl_scan(uint32_t v, uint32_t* total) {
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(x, o, kWave);
        if (lane_id() >= static_cast<uint32_t>(o)) x += y;
    }
    *total = __builtin_amdgcn_readfirstlane(__shfl(x, 63, kWave));
    return x - v;
}

// One step of the segmented scan below: v += the value of the lane DPP control CTRL names, when
// that lane carries the same key (lanes without a source receive v = 0).
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float seg_step(float v, uint32_t key) {
    const int vs = __builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROW_MASK, 0xF, false);
    const int ks = __builtin_amdgcn_update_dpp(-1, static_cast<int>(key), CTRL, ROW_MASK, 0xF, false);
    return static_cast<uint32_t>(ks) == key ? v + __int_as_float(vs) : v;
}

// Inclusive scan of v over runs of equal `key` (runs are contiguous in lane order), in DPP:
// shifts by 1, 2, 4 and 8 within rows of 16 lanes, then the last lane of row 0 (2) into row 1
// (3) and of row 1 into rows 2 and 3.  Each step adds a partial sum only across equal keys, and
// since runs are contiguous the partial it adds covers exactly the earlier lanes of its run.
__device__ __forceinline__ float segmented_scan(float v, uint32_t key) {
    v = seg_step<0x111, 0xF>(v, key);  // row_shr 1
    v = seg_step<0x112, 0xF>(v, key);  // row_shr 2
    v = seg_step<0x114, 0xF>(v, key);  // row_shr 4
    v = seg_step<0x118, 0xF>(v, key);  // row_shr 8
    v = seg_step<0x142, 0xA>(v, key);  // row_bcast 15 into rows 1, 3
    v = seg_step<0x143, 0xC>(v, key);  // row_bcast 31 into rows 2, 3
    return v;
}

// Owner of packed slot g: the largest lane q with off_q <= g (offsets are non-decreasing, so
// this is the pixel holding the slot; six fixed steps keep every lane active for the shuffles).
__device__ __forceinline__ uint32_t packed_owner(uint32_t off, uint32_t g) {
    uint32_t q = 0;
#pragma unroll
    for (int b = 5; b >= 0; --b) {
        const uint32_t cand = q | (1u << b);
        if (__shfl(off, cand, kWave) <= g) q = cand;
    }
    return q;
}

// Task queues: up to kQueues counters, kQueueStride words apart (separate cache lines).  With Q =
// min(kQueues, blocks), block b takes tasks from queue q = b mod Q, which hands out q, q + Q,
// q + 2Q, ...: same-address atomics serialise (about 11 ns each here), so one counter for all
// wavefronts caps the task rate, while blocks are spread over the chip's eight dies in that same
// rotation.  Every queue has at least one block, so every task is taken.
constexpr uint32_t kQueues = 8;
constexpr uint32_t kQueueStride = 32;
constexpr size_t kQueueBytes = size_t(kQueues) * kQueueStride * 4;

__device__ __forceinline__ uint32_t next_task(const Args& a, uint32_t wave_global, uint32_t iter) {
    if (a.dynamic) {
        const uint32_t nq = min(kQueues, gridDim.x);
        const uint32_t q = blockIdx.x % nq;
        uint32_t t = 0;
        if (lane_id() == 0) t = atomicAdd(a.queue + q * kQueueStride, 1u);
        return __builtin_amdgcn_readfirstlane(t) * nq + q;
    }
    return wave_global + iter * a.total_waves;
}

// ------------------------------------------------------------- sampler state ----

template <int D>
struct SamplerLds {
    uint32_t T[D][kWave];  // C_j k for k < 64 (mirrored when scrambling)
    uint32_t Q[D][kQI];    // XOR of columns 6..6+t (mirrored when scrambling)
    uint32_t B0[D];        // C_j begin
    uint32_t kn[D], kc[D], kd[D];
    uint32_t g[D];
};

// Per-wave values of the big pixel being processed.
template <int D>
struct PixelLds {
    uint32_t seed[D], sm[D], shift[D];
    float delta[D];
    uint32_t B[D];       // current per-round index part
    uint32_t gen[4][D];  // lattice: per-pixel random generator of each instance
    uint32_t hshift;     // lattice: the pixel's Hilbert shift of the radical inverse
};

// Per-wave scramble seeds and shifts of the tile's 64 pixels ([dimension][pixel]), formed once
// per tile so that packed pixels do not hash per sample.
template <int D>
struct PackedSeeds {
    uint32_t seed[D][kWave];
    uint32_t shift[D][kWave];
    uint32_t hshift[kWave];  // lattice: Hilbert shift of each pixel
};

// a + b rounded as a separate add: keeps the compiler from contracting it with the product that
// formed b into an FMA, so a sum rounds the same way in every kernel that forms it (the Genz
// kernel's materialised-sample path must reproduce the generating paths bit for bit).
__device__ __forceinline__ float add_nc(float a, float b) {
#pragma clang fp contract(off)
    return a + b;
}

// 2^-e for e >= 0 with the hardware exponential (about 1 ulp); results below 2^-126 may flush
// to zero, which changes a lobe's contribution by less than 1e-38.
__device__ __forceinline__ float exp2_neg(float e) { return __builtin_amdgcn_exp2f(-e); }

__device__ __forceinline__ float pixel_delta(uint32_t kd, uint32_t p) {
    const float u = dev::u32_to_unifloat(dev::pcg_hash(kd ^ p));
    return __fsub_rn(__fmul_rn(0.5f, u), 0.25f);
}

template <int D, uint32_t SK, bool NUS>
__device__ void stage_sampler(SamplerLds<D>& S, const Args& a) {
    const uint32_t tid = threadIdx.x;
    const uint32_t d = min(a.d, static_cast<uint32_t>(D));
    if constexpr (SK == QMC_SAMPLER_SOBOL) {
        for (uint32_t e = tid; e < d * kWave; e += blockDim.x) {
            const uint32_t j = e / kWave, k = e % kWave;
            uint32_t x = 0;
            for (uint32_t b = 0; b < 6; ++b)
                if ((k >> b) & 1u) x ^= a.table[j * 32 + b];
            S.T[j][k] = NUS ? dev::brev(x) : x;
        }
        for (uint32_t e = tid; e < d * kQI; e += blockDim.x) {
            const uint32_t j = e / kQI, t = e % kQI;
            uint32_t x = 0;
            for (uint32_t b = 0; b <= t; ++b) x ^= a.table[j * 32 + 6 + b];
            S.Q[j][t] = NUS ? dev::brev(x) : x;
        }
        for (uint32_t j = tid; j < d; j += blockDim.x) {
            uint32_t x = 0;
            for (uint32_t b = 0; b < 32; ++b)
                if ((a.begin >> b) & 1u) x ^= a.table[j * 32 + b];
            S.B0[j] = NUS ? dev::brev(x) : x;
        }
    }
    for (uint32_t j = tid; j < d; j += blockDim.x) {
        S.kn[j] = dev::pcg_hash(a.seed + 2u * j);
        S.kc[j] = dev::pcg_hash(a.seed + 2u * j + 1u);
        S.kd[j] = dev::pcg_hash(a.pixel_seed + j);
        if constexpr (SK == QMC_SAMPLER_LATTICE) S.g[j] = a.table[j];
    }
}

// Dimensions of a sample generated by one lane: all of them for d <= 32; for d > 32 two lanes
// (l and l + 32) share a sample, each forming one half, so that a lane never holds 64
// coordinates at once.
template <int D>
constexpr int kGen = D > 32 ? 32 : D;

// First dimension this lane generates.
template <int D>
__device__ __forceinline__ uint32_t gen_first_dim() {
    if constexpr (D > 32)
        return (lane_id() >> 5) * 32u;
    else
        return 0u;
}

// Per-dimension Sobol' index part of sample i.  With a per-round base (windows starting on a
// multiple of 64) it is base[j] ^ T[j][k], k = i - begin < 64; otherwise the plain matrix
// product C_j i is formed, looping over index bits outside and dimensions inside so that
// the per-dimension values stay in registers.  Mirrored when scrambling.
template <int D, bool NUS>
__device__ __forceinline__ void index_part(uint32_t (&v)[kGen<D>], const SamplerLds<D>& S, const Args& a, uint32_t i,
                                           uint32_t k, const uint32_t* base, uint32_t j0) {
    constexpr int G = kGen<D>;
    if (base) {
#pragma unroll
        for (int jj = 0; jj < G; ++jj) v[jj] = base[j0 + jj] ^ S.T[j0 + jj][k];
    } else {
#pragma unroll
        for (int jj = 0; jj < G; ++jj) v[jj] = 0u;
        for (uint32_t b = 0; b < 32; ++b) {
            if ((i >> b) & 1u) {
#pragma unroll
                for (int jj = 0; jj < G; ++jj)
                    if (j0 + jj < a.d) v[jj] ^= a.table[(j0 + jj) * 32 + b];
            }
        }
        if constexpr (NUS) {
#pragma unroll
            for (int jj = 0; jj < G; ++jj) v[jj] = dev::brev(v[jj]);
        }
    }
}

// Index of cell (x, y) along the Hilbert curve of the 2^order square: at each scale the quadrant
// (rx, ry) is visited in the order (0,0), (0,1), (1,1), (1,0), i.e. at position (3 rx) ^ ry, and
// the coordinates inside it are mapped to the sub-curve's frame (transposed for ry = 0, and for
// rx = 1 also mirrored), so that consecutive indices are edge-adjacent cells.
__device__ __forceinline__ uint32_t hilbert_index(uint32_t x, uint32_t y, uint32_t order) {
    uint32_t d = 0;
    for (uint32_t h = order; h-- > 0;) {
        const uint32_t rx = (x >> h) & 1u, ry = (y >> h) & 1u;
        d += ((3u * rx) ^ ry) << (2u * h);
        const uint32_t m = (1u << h) - 1u;
        uint32_t xl = x & m, yl = y & m;
        if (!ry) {
            if (rx) {
                xl = m - xl;
                yl = m - yl;
            }
            const uint32_t t = xl;
            xl = yl;
            yl = t;
        }
        x = xl;
        y = yl;
    }
    return d;
}

// floor(2^32 phi_3(n)): the base-3 digits of n mirrored at the point (Sec. 2.2), as the exact
// quotient (reversed digits) * 2^32 / 3^m.
__device__ __forceinline__ uint32_t radical_inverse3_u32(uint32_t n) {
    uint64_t r = 0, pw = 1;
    while (n) {
        const uint32_t q = n / 3u;
        r = r * 3u + (n - 3u * q);
        pw *= 3u;
        n = q;
    }
    return static_cast<uint32_t>((r << 32) / pw);
}

// The shift of pixel p = y * width + x in the radical-inverse domain (Eq. PixelShiftedR1LS).
__device__ __forceinline__ uint32_t pixel_hilbert_shift(const Args& a, uint32_t p) {
    const uint32_t y = p / a.width, x = p - y * a.width;
    return radical_inverse3_u32(hilbert_index(x, y, a.hilbert_order));
}

// Cell of pixel p in the 128 x 128 tables of Sec. 2.6.1: (y mod 128) * 128 + (x mod 128).
__device__ __forceinline__ uint32_t pixel_cell(const Args& a, uint32_t p) {
    const uint32_t y = p / a.width, x = p - y * a.width;
    return ((y & 127u) << 7) | (x & 127u);
}

// Rotation of component j of pixel p: the hashed per-pixel value, or the pixel's entry of the
// table of two-dimensional shifts, shared by every pair of dimensions (entry j mod 2).
__device__ __forceinline__ uint32_t pixel_rotation(const Args& a, uint32_t kc_j, uint32_t j, uint32_t p) {
    if (a.shift_table) return a.shift_table[(j & 1u) * QMC_XOR_TABLE_CELLS + pixel_cell(a, p)];
    return dev::pcg_hash(kc_j ^ p);
}

// Per-pixel random generator component (Alg. 4): H(k + c) | 1 with k = H(H(seed + 2j) ^ p).
__device__ __forceinline__ uint32_t pixel_generator(uint32_t kn_j, uint32_t p, uint32_t c) {
    return dev::pcg_hash(dev::pcg_hash(kn_j ^ p) + c) | 1u;
}

// Components j0 + jj < d (jj < kGen<D>) of sample i of pixel p into x (0 beyond d).
//   base:   per-round index part in LDS (PixelLds::B or SamplerLds::B0); with it, the Sobol'
//           index part is base[j] ^ T[j][k] for k = i - begin mod 64.  NULL: C_j i directly.
//   PX:     per-pixel values of a big pixel; else PK: the tile's per-pixel values, pixel q;
//           both NULL: derive them per lane (hash, or the rotation table of Sec. 2.6.1);
//   valid:  false for lanes past the end of a window, which must not read materialised samples.
template <int D, uint32_t SK, bool NUS, bool SHIFT, bool BACK>
__device__ __forceinline__ void sample_point(float (&x)[kGen<D>], const SamplerLds<D>& S, const PixelLds<D>* PX,
                                             const Args& a, uint32_t p, uint32_t i, uint32_t k,
                                             const uint32_t* base, bool valid, uint32_t j0,
                                             const PackedSeeds<D>* PK = nullptr, uint32_t q = 0) {
    constexpr int G = kGen<D>;
    if constexpr (SK == QMC_SAMPLER_XOR_TABLE) {
        // the pixel's cell of the 128 x 128 tables; stored point (i ^ r_c) mod N, digits ^ s_cj
        const uint32_t c = pixel_cell(a, p);
        const uint32_t idx = valid ? ((i ^ a.xor_reorder[c]) & a.xor_mask) : 0u;
#pragma unroll
        for (int jj = 0; jj < G; ++jj) {
            const uint32_t j = j0 + jj;
            x[jj] = (valid && j < a.d) ? dev::u32_to_unifloat(a.table[uint64_t(j) * a.points_ld + idx] ^
                                                              a.xor_scramble[j * QMC_XOR_TABLE_CELLS + c])
                                       : 0.0f;
        }
    } else if constexpr (SK == QMC_SAMPLER_POINTS) {
        const uint64_t off = valid ? a.offsets[p] + i : 0;
#pragma unroll
        for (int jj = 0; jj < G; ++jj)
            x[jj] = (valid && j0 + jj < a.d) ? a.points[uint64_t(j0 + jj) * a.points_ld + off] : 0.0f;
    } else {
        uint32_t ip[G];
        if constexpr (SK == QMC_SAMPLER_SOBOL) index_part<D, NUS>(ip, S, a, i, k, base, j0);
        // lattice: phi_2 of the index (of the instance's index with four instances), plus the
        // pixel's Hilbert shift; the generator is shared or the pixel's own (Sec. 2.4, Sec. 3)
        const uint32_t inst = (SK == QMC_SAMPLER_LATTICE && a.linst4) ? (i & 3u) : 0u;
        const uint32_t il = (SK == QMC_SAMPLER_LATTICE && a.linst4) ? (i >> 2) : i;
        uint32_t bi = (SK == QMC_SAMPLER_LATTICE) ? dev::brev(BACK ? ~il : il) : 0u;
        if (SK == QMC_SAMPLER_LATTICE && a.lhilbert)
            bi += PX ? PX->hshift : PK ? PK->hshift[q] : pixel_hilbert_shift(a, p);
        // component j before the conversion
        auto component = [&](uint32_t jj, uint32_t j) -> uint32_t {
            uint32_t v;
            if constexpr (SK == QMC_SAMPLER_SOBOL) {
                v = ip[jj];
            } else {
                uint32_t g = S.g[j];
                if (a.lrgen) g = PX ? PX->gen[inst][j] : pixel_generator(S.kn[j], p, inst);
                v = bi * g;
            }
            if constexpr (NUS) {
                uint32_t sd, sm;
                if (PX) {
                    sd = PX->seed[j];
                    sm = PX->sm[j];
                } else if (PK) {
                    sd = PK->seed[j][q];
                    sm = dev::seed_multiplier(sd);
                } else {
                    sd = dev::pcg_hash(S.kn[j] ^ p);
                    sm = dev::seed_multiplier(sd);
                }
                v = dev::nus_from_mirrored(v, sd, sm);
            }
            if constexpr (SHIFT) {
                const uint32_t sh = PX ? PX->shift[j] : PK ? PK->shift[j][q] : pixel_rotation(a, S.kc[j], j, p);
                v = a.sxor ? (v ^ sh) : (v + sh);
            }
            return v;
        };
#pragma unroll
        for (int jj = 0; jj < G; ++jj) {
            const uint32_t j = j0 + jj;
            if constexpr (D > 32) {
                // 64-dimension kernels: unused dimensions are skipped
                x[jj] = 0.0f;
                if (j < a.d) x[jj] = dev::u32_to_unifloat(component(jj, j));
            } else {
                // up to 32 dimensions every component is formed and the unused ones (j >= d,
                // whose table reads stay inside the D-sized arrays) are zeroed by a select: no
                // branch per dimension, which keeps the fused L2 step at four wavefronts per SIMD
                const uint32_t v = component(jj, j);
                x[jj] = j < a.d ? dev::u32_to_unifloat(v) : 0.0f;
            }
        }
    }
}

// ------------------------------------------------------------- tile walker ----
//
// Samples handed to one on_round call: 64 (one per lane), or 32 for d > 32, where lanes l and
// l + 32 form the two halves of sample l.
template <int D>
constexpr uint32_t kRoundSamples = D > 32 ? 32u : kWave;

// Visits every sample of the tile's window in rounds of at most kRoundSamples<D>; the valid
// samples of a round are the prefix r < count, r = lane % kRoundSamples<D>.  Calls, in order:
//   on_big_begin(q)                                 before the rounds of big pixel q;
//   on_round(x, count, q, p, is_big, slot0, i)      for each round (x: this lane's part of
//                                                   its sample, dimensions gen_first_dim() +
//                                                   [0, kGen<D>); q/p: the sample's pixel in
//                                                   the tile / image; slot0: packed slot of
//                                                   sample 0; i: the sample's index);
//   on_big_end(q)                                   after the rounds of big pixel q.
// Packed pixels follow the big ones, in pixel order.  With DELTA the per-pixel integrand
// offsets are added (y = x + delta, rounded to binary32).
template <int D, uint32_t SK, bool NUS, bool SHIFT, bool BACK, bool DELTA, typename BigBegin, typename Round,
          typename BigEnd>
__device__ __forceinline__ void walk_tile(const Args& a, const SamplerLds<D>& S, PixelLds<D>& PX, uint32_t task,
                                          uint32_t n, bool inb, uint32_t off, uint32_t total_small,
                                          BigBegin&& on_big_begin, Round&& on_round, BigEnd&& on_big_end,
                                          PackedSeeds<D>* PK = nullptr) {
    constexpr int G = kGen<D>;
    constexpr uint32_t RS = kRoundSamples<D>;
    const uint32_t lane = lane_id();
    const uint32_t row = RS == kWave ? lane : lane % RS;
    const uint32_t j0 = gen_first_dim<D>();
    const uint32_t p0 = task * kTile;
    // Hilbert-shifted lattice: each lane forms its own pixel's shift once per tile, for the big
    // pixels (read from the owner lane) and the packed ones alike
    uint32_t hs_own = 0;
    if constexpr (SK == QMC_SAMPLER_LATTICE) {
        if (a.lhilbert && p0 + lane < a.num_pixels) hs_own = pixel_hilbert_shift(a, p0 + lane);
    }
    uint64_t bigmask = __ballot(inb && n >= kWave);
    while (bigmask) {
        const uint32_t q = __builtin_ctzll(bigmask);
        bigmask &= bigmask - 1;
        const uint32_t pp = p0 + q;
        const uint32_t nn = __builtin_amdgcn_readfirstlane(__shfl(n, q, kWave));
        if (lane < D && lane < a.d) {
            if constexpr (NUS) {
                const uint32_t sd = dev::pcg_hash(S.kn[lane] ^ pp);
                PX.seed[lane] = sd;
                PX.sm[lane] = dev::seed_multiplier(sd);
            }
            if constexpr (SHIFT) PX.shift[lane] = pixel_rotation(a, S.kc[lane], lane, pp);
            if constexpr (DELTA) PX.delta[lane] = pixel_delta(S.kd[lane], pp);
            if constexpr (SK == QMC_SAMPLER_SOBOL) PX.B[lane] = S.B0[lane];
            if constexpr (SK == QMC_SAMPLER_LATTICE) {
                if (a.lrgen) {
                    for (uint32_t c = 0; c < (a.linst4 ? 4u : 1u); ++c)
                        PX.gen[c][lane] = pixel_generator(S.kn[lane], pp, c);
                }
            }
        }
        if constexpr (SK == QMC_SAMPLER_LATTICE) {
            if (a.lhilbert && lane == 0) PX.hshift = __builtin_amdgcn_readlane(hs_own, q);
        }
        wave_sync();
        on_big_begin(q);
        const uint32_t rounds = (nn + kWave - 1) / kWave;  // blocks of 64 indices
        for (uint32_t r = 0; r < rounds; ++r) {
            // One call per 64 indices, or two (halves of 32 samples) for d > 32; both use the
            // round's index part B, with k & 63 selecting the T entry.
            auto visit = [&](uint32_t kb, uint32_t count, uint32_t t_index) {
                const uint32_t k = kb + row;
                float x[G];
                sample_point<D, SK, NUS, SHIFT, BACK>(x, S, &PX, a, pp, a.begin + k, t_index,
                                                      a.aligned ? PX.B : nullptr, row < count, j0);
                if constexpr (DELTA) {
#pragma unroll
                    for (int jj = 0; jj < G; ++jj) x[jj] = j0 + jj < a.d ? x[jj] + PX.delta[j0 + jj] : 0.0f;
                }
                on_round(x, count, q, pp, true, 0u, a.begin + k);
            };
            if constexpr (RS == kWave) {
                visit(r * kWave, min(nn - r * kWave, kWave), lane);
            } else {
                for (uint32_t part = 0; part < kWave / RS; ++part) {
                    const uint32_t kb = r * kWave + part * RS;
                    if (kb >= nn) break;
                    visit(kb, min(nn - kb, RS), part * RS + row);
                }
            }
            if constexpr (SK == QMC_SAMPLER_SOBOL) {
                if (a.aligned && r + 1 < rounds) {
                    const uint32_t h = (a.begin >> 6) + r;
                    const uint32_t t = min(static_cast<uint32_t>(__builtin_ctz(h + 1u)), kQI - 1);
                    wave_sync();
                    if (lane < D && lane < a.d) PX.B[lane] ^= S.Q[lane][t];
                    wave_sync();
                }
            }
        }
        on_big_end(q);
        wave_sync();
    }

    if (PK && total_small) {
        // every lane hashes its own pixel's values (pixels without packed samples are unused)
        for (uint32_t j = 0; j < a.d && j < D; ++j) {
            if constexpr (NUS) PK->seed[j][lane] = dev::pcg_hash(S.kn[j] ^ (p0 + lane));
            if constexpr (SHIFT) PK->shift[j][lane] = pixel_rotation(a, S.kc[j], j, p0 + lane);
        }
        if constexpr (SK == QMC_SAMPLER_LATTICE) {
            if (a.lhilbert) PK->hshift[lane] = hs_own;
        }
        wave_sync();
    }
    for (uint32_t sb = 0; sb < total_small; sb += RS) {
        const uint32_t g = sb + row;
        const uint32_t count = min(total_small - sb, RS);
        const bool valid = row < count;
        const uint32_t qo = packed_owner(off, g);
        const uint32_t offq = __shfl(off, qo, kWave);
        const uint32_t q = valid ? qo : 0u;
        const uint32_t pp = p0 + q;
        const uint32_t k = valid ? g - offq : 0u;
        float x[G];
        sample_point<D, SK, NUS, SHIFT, BACK>(x, S, nullptr, a, pp, a.begin + k, k & (kWave - 1),
                                              a.aligned ? S.B0 : nullptr, valid, j0, PK, q);
        if constexpr (DELTA) {
#pragma unroll
            for (int jj = 0; jj < G; ++jj)
                x[jj] = j0 + jj < a.d ? x[jj] + pixel_delta(S.kd[j0 + jj], pp) : 0.0f;
        }
        on_round(x, count, q, pp, false, sb, a.begin + k);
    }
}

// Per-tile bookkeeping common to every consumer: window counts and packed offsets.
struct TileInfo {
    uint32_t p;      // this lane's pixel
    bool inb;        // p < num_pixels
    uint32_t n;      // samples of p in the window
    uint32_t ns;     // n if p is packed, else 0
    uint32_t off;    // packed slot of p's first sample
    uint32_t total;  // packed slots in the tile
};

__device__ __forceinline__ TileInfo tile_info(const Args& a, uint32_t task) {
    TileInfo t;
    t.p = task * kTile + lane_id();
    t.inb = t.p < a.num_pixels;
    const uint32_t N = t.inb ? a.counts[t.p] : 0u;
    const uint32_t hi = min(N, a.end);
    t.n = hi > a.begin ? hi - a.begin : 0u;
    t.ns = (t.inb && t.n < kWave) ? t.n : 0u;
    t.off = wave_excl_scan(t.ns, &t.total);
    return t;
}

// Stores the pixel's running sum and mean given its total count N.
__device__ __forceinline__ void write_pixel_n(const Args& a, uint32_t p, float window_sum, uint32_t N) {
    float total = window_sum;
    if (a.sums) {
        total = a.sums[p] + window_sum;
        a.sums[p] = total;
    }
    if (a.means) a.means[p] = N ? total / static_cast<float>(N) : 0.0f;
}

__device__ __forceinline__ void write_pixel(const Args& a, uint32_t p, float window_sum) {
    write_pixel_n(a, p, window_sum, a.counts[p]);
}

// Runs body(task) for every task this wavefront obtains.
template <typename F>
__device__ __forceinline__ void for_each_task(const Args& a, F&& body) {
    const uint32_t wave_global = blockIdx.x * kWavesPerBlock + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    for (uint32_t it = 0;; ++it) {
        const uint32_t task = next_task(a, wave_global, it);
        if (task >= a.num_tasks) break;
        body(task);
    }
}

// Adds v exactly into accumulator entry e (its kAccWords words in this block's copy).  The
// integer m 2^(pos mod 32), m the significand and pos = max(exponent field, 1) - 1, spans the
// 32-bit digit positions k = pos / 32 and k + 1; both digits carry the sign of v.  Infinities
// and NaNs add 1 to the last word instead, which makes the result NaN.  Branch-free: zeros add
// zero digits.
__device__ __forceinline__ void acc_add(const Args& a, uint32_t e, float v) {
    unsigned long long* w = a.acc + (uint64_t(blockIdx.x % kAccCopies) * a.n_row + e) * kAccWords;
    const uint32_t bits = __float_as_uint(v);
    const uint32_t ex = (bits >> 23) & 0xFFu;
    const uint32_t m = (bits & 0x7FFFFFu) | (ex ? 0x800000u : 0u);
    const uint32_t pos = ex ? ex - 1u : 0u;
    const uint32_t sh = pos & 31u;
    const uint32_t lo = m << sh, hi = (m >> 1) >> (31u - sh);
    const bool finite = ex != 0xFFu;
    const bool neg = (bits >> 31) != 0;
    const uint32_t k = finite ? (pos >> 5) : kAccWords - 2;
    const unsigned long long dlo = finite ? (neg ? 0ull - lo : static_cast<unsigned long long>(lo)) : 0ull;
    const unsigned long long dhi = finite ? (neg ? 0ull - hi : static_cast<unsigned long long>(hi)) : 1ull;
    atomicAdd(&w[k], dlo);
    atomicAdd(&w[k + 1], dhi);
}

// ------------------------------------------------------------ Genz forward ----
//
// Genz product f(x) = exp(-sum_{j<4} a_j^2 (x_j - u_j)^2) * cos(2 pi u_4 + sum_{j>=4} a_j x_j),
// evaluated as exp2(-sum (c_j (x_j - u_j))^2) with c_j = a_j sqrt(log2 e), and the phase in
// turns, phi = u_4 + sum_{j>=4} (a_j / 2 pi) x_j, reduced to [-1/2, 1/2] before the hardware
// cosine (which takes its argument in turns).  Generated samples enter as X = x 2^32 (the float
// before the final scaling of the conversion) with U = u 2^32, C = c 2^-32 and B = b 2^-32: every
// operation then rounds exactly as it does on x (scaling by a power of two is exact), so the
// result equals that of the materialised samples bit for bit, one multiply per dimension sooner.
//
// Work decomposition: every pixel is integrated by one lane, which keeps the pixel's seeds,
// rotations, constants and sum in registers.  Three small launches sort the pixels into buckets
// (exact counts below 64, counts within a factor of two above), and a task is 64 pixels of one
// bucket, one per lane, all lanes stepping through k = 0, 1, ... together (a lane adds only its
// own n samples).  The sample index i = begin + k is then the same in every lane, so the Sobol'
// index part C_j(i) = C_j(i - i mod 64) ^ C_j(i mod 64) comes from tables through the scalar
// cache, updated once per 64 steps, and the lattice's phi_2(i) is a scalar value; only the
// per-pixel scramble, rotation, conversion and the integrand remain per lane.  Each pixel's sum
// is formed in sample order by one lane, so results depend neither on the order inside a bucket
// nor on the schedule.

__device__ __forceinline__ uint32_t window_count(const Args& a, uint32_t N) {
    const uint32_t hi = min(N, a.end);
    return hi > a.begin ? hi - a.begin : 0u;
}

// Bucket of a pixel with n >= 1 samples in the window: n itself below 64, else 64 + floor(log2(n /
// 64)), so buckets 1 .. 89; tasks take the buckets from 89 down (the longest first).
constexpr uint32_t kBuckets = 90;
__device__ __forceinline__ uint32_t genz_bucket(uint32_t n) {
    return n < kWave ? n : kWave + 31u - static_cast<uint32_t>(__builtin_clz(n >> 6));
}

// Per-pixel constants; SCALED: for samples X = x 2^32 (see above).
struct GenzPixel {
    float u[4], c[4], phi0, b[4];
    template <bool SCALED>
    __device__ __forceinline__ void load(const Args& a, uint32_t p) {
        const float* pp = a.pixel_params + uint64_t(p) * 16;
        constexpr float kSqrtLog2e = 1.2011224087864498f;  // sqrt(log2(e))
        constexpr float kInv2Pi = 0.15915494309189535f;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            u[j] = pp[j];
            c[j] = pp[8 + j] * kSqrtLog2e;
            b[j] = pp[12 + j] * kInv2Pi;
            if constexpr (SCALED) {
                u[j] *= 0x1p32f;
                c[j] *= 0x1p-32f;
                b[j] *= 0x1p-32f;
            }
        }
        phi0 = pp[4];
    }
    __device__ __forceinline__ float eval(const float (&x)[8]) const {
        float e = 0.0f;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const float t = c[j] * (x[j] - u[j]);
            e = fmaf(t, t, e);
        }
        float ph = phi0;
#pragma unroll
        for (int j = 0; j < 4; ++j) ph = fmaf(b[j], x[4 + j], ph);
        ph -= rintf(ph);
        return exp2_neg(e) * __builtin_amdgcn_cosf(ph);
    }
};

// Reads through the scalar cache: p must be the same in every lane.
typedef const __attribute__((address_space(4))) uint32_t scalar_u32;
__device__ __forceinline__ uint32_t sload(const uint32_t* p) { return *(const scalar_u32*)p; }

// Sobol' tables of the Genz kernel, written before the integration launch (genz_tables):
// T[l][j] = C_j l for l < 64, Q[t][j] = XOR of columns 6 .. 6 + t (what C_j changes by when
// index bits 6 .. 6 + t flip), H0[j] = C_j(begin - begin mod 64); mirrored when scrambling.
// Word offsets:
constexpr uint32_t kTabT = 0, kTabQ = 512, kTabH0 = kTabQ + kQI * 8, kTabWords = kTabH0 + 8;

// Wave-uniform keys of the per-pixel hashes and the shared lattice generator (dimensions 0..7),
// formed from the launch arguments in scalar registers.
struct GenzKeys {
    uint32_t kn[8], kc[8], g[8];
    __device__ __forceinline__ void init(const Args& a) {
#pragma unroll
        for (uint32_t j = 0; j < 8; ++j) {
            kn[j] = dev::pcg_hash(a.seed + 2u * j);
            kc[j] = dev::pcg_hash(a.seed + 2u * j + 1u);
            g[j] = a.skind == QMC_SAMPLER_LATTICE ? sload(a.table + j) : 0u;
        }
    }
};

// Sampler state of one pixel (dimensions 0..7), held by its lane: NUS seeds and their
// multipliers, rotations, the lattice's Hilbert shift and generators, the XOR table sampler's
// reorder entry and digit scrambles, or the materialised samples' offset.
template <uint32_t SK, bool NUS, bool SHIFT>
struct GenzSampler {
    uint32_t seed[8], sm[8], shift[8];
    uint32_t hs;
    uint32_t gen[4][8];
    uint32_t rc, scr[8];
    uint64_t off;
    __device__ __forceinline__ void init(const GenzKeys& K, const Args& a, uint32_t p) {
#pragma unroll
        for (uint32_t j = 0; j < 8; ++j) {
            if constexpr (NUS) {
                seed[j] = dev::pcg_hash(K.kn[j] ^ p);
                sm[j] = dev::seed_multiplier(seed[j]);
            }
            if constexpr (SHIFT) shift[j] = pixel_rotation(a, K.kc[j], j, p);
        }
        if constexpr (SK == QMC_SAMPLER_LATTICE) {
            hs = a.lhilbert ? pixel_hilbert_shift(a, p) : 0u;
            if (a.lrgen) {
#pragma unroll
                for (uint32_t c = 0; c < 4; ++c)
#pragma unroll
                    for (uint32_t j = 0; j < 8; ++j) gen[c][j] = (c == 0 || a.linst4) ? pixel_generator(K.kn[j], p, c) : 0u;
            }
        }
        if constexpr (SK == QMC_SAMPLER_XOR_TABLE) {
            const uint32_t c = pixel_cell(a, p);
            rc = a.xor_reorder[c];
#pragma unroll
            for (uint32_t j = 0; j < 8; ++j) scr[j] = a.xor_scramble[j * QMC_XOR_TABLE_CELLS + c];
        }
        if constexpr (SK == QMC_SAMPLER_POINTS) off = a.offsets[p];
    }
};

// Randomisation and conversion of a generated component v (X = x 2^32); SX: rotation by XOR
// instead of addition.
template <bool NUS, bool SHIFT, bool SX>
__device__ __forceinline__ float genz_finish(uint32_t v, uint32_t seed, uint32_t sm, uint32_t shift) {
    if constexpr (NUS) v = dev::nus_from_mirrored(v, seed, sm);
    if constexpr (SHIFT) v = SX ? (v ^ shift) : (v + shift);
    return dev::u32_to_unifloat_x32(v);
}

// Sample i = begin + k of the lane's pixel (k, i and ip uniform): X = x 2^32 for generated
// samples, x itself for materialised ones.  ip: the Sobol' index parts C_j(i); lanes past
// their own n (valid false) must not read materialised samples.
template <uint32_t SK, bool NUS, bool SHIFT, bool BACK, bool SX, uint32_t INST>
__device__ __forceinline__ void genz_sample(float (&X)[8], const GenzSampler<SK, NUS, SHIFT>& g, const GenzKeys& K,
                                            const Args& a, uint32_t i, const uint32_t (&ip)[8], bool valid) {
    if constexpr (SK == QMC_SAMPLER_SOBOL) {
#pragma unroll
        for (int j = 0; j < 8; ++j) X[j] = genz_finish<NUS, SHIFT, SX>(ip[j], g.seed[j], g.sm[j], g.shift[j]);
    } else if constexpr (SK == QMC_SAMPLER_LATTICE) {
        const uint32_t il = a.linst4 ? (i >> 2) : i;
        const uint32_t bi = dev::brev(BACK ? ~il : il) + g.hs;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const uint32_t gj = a.lrgen ? g.gen[INST][j] : K.g[j];
            X[j] = genz_finish<false, SHIFT, SX>(bi * gj, 0u, 0u, g.shift[j]);
        }
    } else if constexpr (SK == QMC_SAMPLER_XOR_TABLE) {
        const uint32_t idx = (i ^ g.rc) & a.xor_mask;
#pragma unroll
        for (int j = 0; j < 8; ++j)
            X[j] = dev::u32_to_unifloat_x32(a.table[uint64_t(j) * a.points_ld + idx] ^ g.scr[j]);
    } else {
#pragma unroll
        for (int j = 0; j < 8; ++j) X[j] = valid ? a.points[uint64_t(j) * a.points_ld + g.off + i] : 0.0f;
    }
}

// Integrates the lane's pixel p (n samples in the window) in a wavefront whose lanes step
// through k < nmax together (nmax: the largest n of the task, uniform).
template <uint32_t SK, bool NUS, bool SHIFT, bool BACK, bool SX>
__device__ __forceinline__ float genz_pixel(const GenzKeys& K, const Args& a, uint32_t p, uint32_t n, uint32_t nmax) {
    constexpr bool kScaled = SK != QMC_SAMPLER_POINTS;
    GenzPixel gp;
    gp.load<kScaled>(a, p);
    GenzSampler<SK, NUS, SHIFT> g;
    g.init(K, a, p);
    float acc = 0.0f;
    if constexpr (SK == QMC_SAMPLER_POINTS) {
        // Chunks of 32 samples, dimension by dimension: the lane reads 128 consecutive bytes of a
        // dimension at a time (whole cache lines, not 16 bytes of 64 lines that must stay cached
        // until the lane returns), keeping the exponent and phase sums of the chunk's samples.
        // Per sample the operations and their order are those of GenzPixel::eval.
        constexpr uint32_t kC = 32;
        const float* base = a.points + g.off + a.begin;
        for (uint32_t k0 = 0; k0 < nmax; k0 += kC) {
            if (k0 + kC <= n) {
                float e[kC], ph[kC];
#pragma unroll
                for (uint32_t t = 0; t < kC; ++t) {
                    e[t] = 0.0f;
                    ph[t] = gp.phi0;
                }
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const float* row = base + uint64_t(j) * a.points_ld + k0;
#pragma unroll
                    for (uint32_t q = 0; q < kC / 4; ++q) {
                        const f32x4 v = *reinterpret_cast<const f32x4_a4*>(row + 4 * q);
#pragma unroll
                        for (uint32_t r = 0; r < 4; ++r) {
                            const uint32_t t = 4 * q + r;
                            if (j < 4) {
                                const float d = gp.c[j] * (v[r] - gp.u[j]);
                                e[t] = fmaf(d, d, e[t]);
                            } else {
                                ph[t] = fmaf(gp.b[j - 4], v[r], ph[t]);
                            }
                        }
                    }
                    // one dimension's loads in flight at a time
                    asm volatile("" ::: "memory");
                }
#pragma unroll
                for (uint32_t t = 0; t < kC; ++t) {
                    const float w = ph[t] - rintf(ph[t]);
                    acc = add_nc(acc, exp2_neg(e[t]) * __builtin_amdgcn_cosf(w));
                }
            } else {
                // the pixel's last, partial chunk: sample by sample
                for (uint32_t k = k0; k < n; ++k) {
                    float X[8];
#pragma unroll
                    for (int j = 0; j < 8; ++j) X[j] = base[uint64_t(j) * a.points_ld + k];
                    acc = add_nc(acc, gp.eval(X));
                }
            }
        }
        return acc;
    }
    if constexpr (SK == QMC_SAMPLER_XOR_TABLE) {
        // Samples i = begin + k in aligned groups of four: the table indices (i ^ rc) & mask of
        // such a group are the four entries of one aligned group of four (N >= 4), entry t ^ (rc & 3)
        // holding sample i + t, so one 16-byte load per dimension fetches them.  The values are
        // summed in sample order.
        uint32_t k = 0;
        const auto single = [&](uint32_t kk) {
            float X[8];
            const uint32_t none[8] = {};
            genz_sample<SK, NUS, SHIFT, BACK, SX, 0>(X, g, K, a, a.begin + kk, none, true);
            const float f = gp.eval(X);
            if (kk < n) acc = add_nc(acc, f);
        };
        if (a.xor_mask >= 3u) {
            const uint32_t head = min(nmax, (4u - (a.begin & 3u)) & 3u);
            for (; k < head; ++k) single(k);
            const bool b0 = (g.rc & 1u) != 0, b1 = (g.rc & 2u) != 0;
            for (; k + 4 <= nmax; k += 4) {
                const uint32_t idx = ((a.begin + k) ^ g.rc) & a.xor_mask & ~3u;
                u32x4_a4 w[8];
#pragma unroll
                for (int j = 0; j < 8; ++j)
                    w[j] = *reinterpret_cast<const u32x4_a4*>(a.table + uint64_t(j) * a.points_ld + idx);
                float f[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    float X[8];
#pragma unroll
                    for (int j = 0; j < 8; ++j) X[j] = dev::u32_to_unifloat_x32(w[j][r] ^ g.scr[j]);
                    f[r] = gp.eval(X);
                }
                // s[t] = f[t ^ (rc & 3)]
                const float g0 = b0 ? f[1] : f[0], g1 = b0 ? f[0] : f[1], g2 = b0 ? f[3] : f[2], g3 = b0 ? f[2] : f[3];
                const float s0 = b1 ? g2 : g0, s1 = b1 ? g3 : g1, s2 = b1 ? g0 : g2, s3 = b1 ? g1 : g3;
                if (k < n) acc = add_nc(acc, s0);
                if (k + 1 < n) acc = add_nc(acc, s1);
                if (k + 2 < n) acc = add_nc(acc, s2);
                if (k + 3 < n) acc = add_nc(acc, s3);
            }
        }
        for (; k < nmax; ++k) single(k);
        return acc;
    }
    // Sobol' index part of step k: h = C_j(i - i mod 64) (uniform, advanced once per 64 indices)
    // XOR T[i mod 64][j] (one scalar load of 32 bytes)
    uint32_t h[8];
    if constexpr (SK == QMC_SAMPLER_SOBOL) {
#pragma unroll
        for (int j = 0; j < 8; ++j) h[j] = sload(a.genz_tab + kTabH0 + j);
    }
    uint32_t k0 = 0;
    if constexpr (SK == QMC_SAMPLER_SOBOL) {
        // two samples per step: both index parts first (scalar work and its branch), then the two
        // samples' vector work in one block
        for (; k0 + 2 <= nmax; k0 += 2) {
            uint32_t ipa[8], ipb[8];
            const uint32_t i = a.begin + k0;
#pragma unroll
            for (int j = 0; j < 8; ++j) ipa[j] = h[j] ^ sload(a.genz_tab + kTabT + (i & 63u) * 8 + j);
            if (((i + 1u) & 63u) == 0u) {
                const uint32_t t = min(static_cast<uint32_t>(__builtin_ctz((i + 1u) >> 6)), kQI - 1);
#pragma unroll
                for (int j = 0; j < 8; ++j) h[j] ^= sload(a.genz_tab + kTabQ + t * 8 + j);
            }
#pragma unroll
            for (int j = 0; j < 8; ++j) ipb[j] = h[j] ^ sload(a.genz_tab + kTabT + ((i + 1u) & 63u) * 8 + j);
            if (((i + 2u) & 63u) == 0u) {
                const uint32_t t = min(static_cast<uint32_t>(__builtin_ctz((i + 2u) >> 6)), kQI - 1);
#pragma unroll
                for (int j = 0; j < 8; ++j) h[j] ^= sload(a.genz_tab + kTabQ + t * 8 + j);
            }
            float Xa[8], Xb[8];
            genz_sample<SK, NUS, SHIFT, BACK, SX, 0>(Xa, g, K, a, i, ipa, true);
            genz_sample<SK, NUS, SHIFT, BACK, SX, 0>(Xb, g, K, a, i + 1u, ipb, true);
            const float fa = gp.eval(Xa);
            const float fb = gp.eval(Xb);
            if (k0 < n) acc = add_nc(acc, fa);
            if (k0 + 1 < n) acc = add_nc(acc, fb);
        }
    }
    for (uint32_t k = k0; k < nmax; ++k) {
        const uint32_t i = a.begin + k;
        uint32_t ip[8];
        if constexpr (SK == QMC_SAMPLER_SOBOL) {
#pragma unroll
            for (int j = 0; j < 8; ++j) ip[j] = h[j] ^ sload(a.genz_tab + kTabT + (i & 63u) * 8 + j);
            if (((i + 1u) & 63u) == 0u) {
                const uint32_t t = min(static_cast<uint32_t>(__builtin_ctz((i + 1u) >> 6)), kQI - 1);
#pragma unroll
                for (int j = 0; j < 8; ++j) h[j] ^= sload(a.genz_tab + kTabQ + t * 8 + j);
            }
        }
        float X[8];
        if (SK == QMC_SAMPLER_LATTICE && a.lrgen && a.linst4) {
            // four superimposed instances: sample i belongs to instance i mod 4 (uniform)
            switch (i & 3u) {
                case 0: genz_sample<SK, NUS, SHIFT, BACK, SX, 0>(X, g, K, a, i, ip, true); break;
                case 1: genz_sample<SK, NUS, SHIFT, BACK, SX, 1>(X, g, K, a, i, ip, true); break;
                case 2: genz_sample<SK, NUS, SHIFT, BACK, SX, 2>(X, g, K, a, i, ip, true); break;
                default: genz_sample<SK, NUS, SHIFT, BACK, SX, 3>(X, g, K, a, i, ip, true); break;
            }
        } else {
            genz_sample<SK, NUS, SHIFT, BACK, SX, 0>(X, g, K, a, i, ip, true);
        }
        const float f = gp.eval(X);
        if (k < n) acc = add_nc(acc, f);
    }
    return acc;
}

// Bucketing, without atomics and in a fixed order.  Each bucketing wavefront covers 1024
// consecutive pixels.  (1) genz_bucket_count writes each wavefront's bucket sizes to
// bucket_wave[b][w]; (2) genz_bucket_scan turns each bucket's row into exclusive prefix sums over
// the wavefronts and stores the bucket's total; (3) genz_bucket_fill writes the pixels to
// bucket_list, bucket b starting at sum_{b' > b} total[b'], within a bucket by wavefront and then
// pixel order; it also writes the results of pixels without samples in the window, which no task
// visits.  A lane keeps the values of buckets lane and lane + 64.
constexpr uint32_t kBucketPixels = 1024;  // pixels per bucketing wavefront

// Calls visit(b, same) for each distinct bucket b among the 64 pixels p0 + lane (same: the lanes
// holding a pixel of bucket b).
template <typename F>
__device__ __forceinline__ void group_buckets(const Args& a, uint32_t p0, uint32_t* n_out, F&& visit) {
    const uint32_t p = p0 + lane_id();
    const uint32_t n = p < a.num_pixels ? window_count(a, a.counts[p]) : 0u;
    *n_out = n;
    const uint32_t b = n ? genz_bucket(n) : 0u;
    bool pend = n != 0;
    uint64_t mask = __ballot(pend);
    while (mask) {
        const uint32_t b0 = __builtin_amdgcn_readlane(b, __builtin_ctzll(mask));
        const uint64_t same = __ballot(pend && b == b0);
        visit(b0, same);
        if (b == b0) pend = false;
        mask &= ~same;
    }
}

// The Sobol' tables of the Genz kernel (see kTabT), by the first block of the counting launch.
__device__ void genz_tables(const Args& a) {
    const bool nus = (a.sflags & QMC_PIXEL_NUS) != 0;
    for (uint32_t e = threadIdx.x; e < kTabWords; e += blockDim.x) {
        uint32_t j, lo = 0, hi, idx;  // columns [lo, hi) selected by the bits of idx
        if (e < kTabQ) {
            j = e & 7u;
            idx = e >> 3;
            hi = 6;
        } else if (e < kTabH0) {
            j = (e - kTabQ) & 7u;
            lo = 6;
            hi = 7 + (e - kTabQ) / 8;
            idx = 0xFFFFFFFFu;
        } else {
            j = e - kTabH0;
            idx = a.begin & ~63u;
            hi = 32;
        }
        uint32_t x = 0;
        for (uint32_t bt = lo; bt < hi; ++bt)
            if ((idx >> bt) & 1u) x ^= a.table[j * 32 + bt];
        a.genz_tab[e] = nus ? dev::brev(x) : x;
    }
}

__global__ __launch_bounds__(256) void genz_bucket_count(Args a) {
    if (blockIdx.x == 0 && a.skind == QMC_SAMPLER_SOBOL) genz_tables(a);
    const uint32_t lane = lane_id();
    const uint32_t w = blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
    if (w >= a.bucket_waves) return;
    uint32_t cnt0 = 0, cnt1 = 0;  // buckets lane and lane + 64
    for (uint32_t r = 0; r < kBucketPixels / kWave; ++r) {
        uint32_t n;
        group_buckets(a, w * kBucketPixels + r * kWave, &n, [&](uint32_t b0, uint64_t same) {
            const uint32_t c = static_cast<uint32_t>(__popcll(same));
            if (lane == (b0 & 63u)) {
                if (b0 < kWave)
                    cnt0 += c;
                else
                    cnt1 += c;
            }
        });
    }
    a.bucket_wave[uint64_t(lane) * a.bucket_waves + w] = cnt0;
    if (lane + kWave < kBuckets) a.bucket_wave[uint64_t(lane + kWave) * a.bucket_waves + w] = cnt1;
}

// One block per bucket: exclusive prefix sums of the bucket's per-wavefront counts, in place.
__global__ __launch_bounds__(1024) void genz_bucket_scan(Args a) {
    __shared__ uint32_t part[1024];
    uint32_t* row = a.bucket_wave + uint64_t(blockIdx.x) * a.bucket_waves;
    const uint32_t t = threadIdx.x;
    const uint32_t per = (a.bucket_waves + 1023) / 1024;  // consecutive entries per thread
    uint32_t sum = 0;
    for (uint32_t k = 0; k < per; ++k) {
        const uint32_t i = t * per + k;
        if (i < a.bucket_waves) sum += row[i];
    }
    part[t] = sum;
    __syncthreads();
    for (uint32_t o = 1; o < 1024; o <<= 1) {
        const uint32_t add = t >= o ? part[t - o] : 0u;
        __syncthreads();
        part[t] += add;
        __syncthreads();
    }
    uint32_t run = part[t] - sum;
    for (uint32_t k = 0; k < per; ++k) {
        const uint32_t i = t * per + k;
        if (i < a.bucket_waves) {
            const uint32_t v = row[i];
            row[i] = run;
            run += v;
        }
    }
    if (t == 1023) a.bucket_total[blockIdx.x] = part[1023];
}

// Inclusive suffix sum over the lanes (lane l receives sum_{m >= l} v_m).
__device__ __forceinline__ uint32_t wave_suffix_sum(uint32_t v) {
    const uint32_t lane = lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t u = __shfl_down(v, o, kWave);
        if (lane + o < 64) v += u;
    }
    return v;
}

__global__ __launch_bounds__(256) void genz_bucket_fill(Args a) {
    const uint32_t lane = lane_id();
    const uint32_t w = blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
    if (w >= a.bucket_waves) return;
    // where this wavefront's entries of buckets lane (base0) and lane + 64 (base1) begin
    const uint32_t t0 = lane >= 1 ? a.bucket_total[lane] : 0u;
    const uint32_t t1 = lane + kWave < kBuckets ? a.bucket_total[lane + kWave] : 0u;
    const uint32_t s1 = wave_suffix_sum(t1);
    const uint32_t all1 = __builtin_amdgcn_readfirstlane(s1);  // every bucket >= 64
    const uint32_t s0 = wave_suffix_sum(t0);
    uint32_t base0 = a.bucket_wave[uint64_t(lane) * a.bucket_waves + w] + (s0 - t0) + all1;
    uint32_t base1 = lane + kWave < kBuckets ? a.bucket_wave[uint64_t(lane + kWave) * a.bucket_waves + w] + (s1 - t1)
                                              : 0u;
    for (uint32_t r = 0; r < kBucketPixels / kWave; ++r) {
        const uint32_t p0 = w * kBucketPixels + r * kWave;
        uint32_t n;
        group_buckets(a, p0, &n, [&](uint32_t b0, uint64_t same) {
            const uint32_t l0 = b0 & 63u;
            const uint32_t pos = b0 < kWave ? __builtin_amdgcn_readlane(base0, l0) : __builtin_amdgcn_readlane(base1, l0);
            if ((same >> lane) & 1u)
                a.bucket_list[pos + static_cast<uint32_t>(__popcll(same & ((uint64_t(1) << lane) - 1u)))] = p0 + lane;
            if (lane == l0) {
                if (b0 < kWave)
                    base0 += static_cast<uint32_t>(__popcll(same));
                else
                    base1 += static_cast<uint32_t>(__popcll(same));
            }
        });
        const uint32_t p = p0 + lane;
        if (p < a.num_pixels && n == 0) write_pixel_n(a, p, 0.0f, a.counts[p]);
    }
}

// Materialised samples of a task's pixels with 64 or more samples: the wavefront takes the pixels
// one at a time, a lane per sample, so that each load instruction reads 256 consecutive bytes of a
// dimension (one lane per pixel reads eight dimension rows per pixel, 512 scattered streams per
// wavefront).  The values are summed in sample order, one lane's value after the other, so the
// result equals the generating paths' bit for bit.
__device__ void genz_points_by_pixel(const Args& a, uint32_t p, uint32_t n, uint32_t N, bool valid) {
    const uint32_t lane = lane_id();
    uint64_t todo = __ballot(valid);
    while (todo) {
        const uint32_t r = static_cast<uint32_t>(__builtin_ctzll(todo));
        todo &= todo - 1;
        const uint32_t pr = __builtin_amdgcn_readlane(p, r);
        const uint32_t nr = __builtin_amdgcn_readlane(n, r);
        const uint32_t Nr = __builtin_amdgcn_readlane(N, r);
        GenzPixel gp;
        gp.load<false>(a, pr);
        const float* base = a.points + a.offsets[pr] + a.begin;
        float acc = 0.0f;
        for (uint32_t k0 = 0; k0 < nr; k0 += kWave) {
            const uint32_t k = k0 + lane;
            float X[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) X[j] = k < nr ? base[uint64_t(j) * a.points_ld + k] : 0.0f;
            const float f = gp.eval(X);
            const uint32_t cnt = min(kWave, nr - k0);
            for (uint32_t t = 0; t < cnt; ++t)
                acc = add_nc(acc, __uint_as_float(__builtin_amdgcn_readlane(__float_as_uint(f), t)));
        }
        if (lane == 0) write_pixel_n(a, pr, acc, Nr);
    }
}

template <uint32_t SK, bool NUS, bool SHIFT, bool BACK>
__global__ __launch_bounds__(kBlock) void genz_fwd(Args a) {
    // Task table in processing order (position q holds bucket 89 - q): first chunk and first list
    // entry of each bucket, and the bucket's size.
    __shared__ uint32_t cs[kBuckets], ls[kBuckets], sz[kBuckets];
    if (threadIdx.x < kWave) {
        const uint32_t lane = threadIdx.x;
        // lane l: positions l and l + 64 (buckets 89 - l and 25 - l)
        const uint32_t h0 = a.bucket_total[kBuckets - 1 - lane];
        const uint32_t h1 = lane + kWave < kBuckets - 1 ? a.bucket_total[kBuckets - 1 - kWave - lane] : 0u;
        uint32_t c0tot, l0tot, dummy;
        const uint32_t c0 = wave_excl_scan((h0 + kWave - 1) / kWave, &c0tot);
        const uint32_t l0 = wave_excl_scan(h0, &l0tot);
        const uint32_t c1 = wave_excl_scan((h1 + kWave - 1) / kWave, &dummy) + c0tot;
        const uint32_t l1 = wave_excl_scan(h1, &dummy) + l0tot;
        cs[lane] = c0;
        ls[lane] = l0;
        sz[lane] = h0;
        if (lane + kWave < kBuckets) {
            cs[lane + kWave] = c1;
            ls[lane + kWave] = l1;
            sz[lane + kWave] = h1;
        }
    }
    __syncthreads();
    GenzKeys K;
    K.init(a);
    const uint32_t lane = lane_id();
    const uint32_t last = kBuckets - 2;  // position of bucket 1
    const uint32_t ntasks = cs[last] + (sz[last] + kWave - 1) / kWave;
    const uint32_t wave_global = blockIdx.x * kWavesPerBlock + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    for (uint32_t iter = 0;; ++iter) {
        const uint32_t t = next_task(a, wave_global, iter);
        if (t >= ntasks) break;
        // the last position with cs <= t (positions of empty buckets share the next one's cs)
        uint32_t q = 0;
        for (uint32_t step = 64; step; step >>= 1)
            if (q + step <= last && cs[q + step] <= t) q += step;
        const uint32_t first = (t - cs[q]) * kWave;
        const bool valid = first + lane < sz[q];
        const uint32_t p = valid ? a.bucket_list[ls[q] + first + lane] : 0u;
        const uint32_t N = valid ? a.counts[p] : 0u;
        const uint32_t n = valid ? window_count(a, N) : 0u;
        const uint32_t b = kBuckets - 1 - q;
        if constexpr (SK == QMC_SAMPLER_POINTS) {
            if (b >= kWave) {
                genz_points_by_pixel(a, p, n, N, valid);
                continue;
            }
        }
        // exact counts below 64; above, the task steps to its largest count
        uint32_t nmax = b;
        if (b >= kWave) {
            uint32_t m = n;
#pragma unroll
            for (int o = 32; o >= 1; o >>= 1) m = max(m, static_cast<uint32_t>(__shfl_xor(m, o, kWave)));
            nmax = __builtin_amdgcn_readfirstlane(m);
        }
        if (valid) {
            const float s = (SHIFT && a.sxor) ? genz_pixel<SK, NUS, SHIFT, BACK, true>(K, a, p, n, nmax)
                                              : genz_pixel<SK, NUS, SHIFT, BACK, false>(K, a, p, n, nmax);
            write_pixel_n(a, p, s, N);
        }
    }
}

// ----------------------------------------------------- lobes: shared layout ----

// Lane -> (half h, lobe slot).  DH dimensions per lane, H = D / DH halves, LPG lobes per group.
template <int D>
struct LobeLayout {
    static constexpr int DH = D > 32 ? 32 : D;
    static constexpr int H = D / DH;
    static constexpr uint32_t LPG = kWave / H;
};

// Staged samples of one round (kRoundSamples<D> rows).
template <int D>
struct StageLds {
    static constexpr uint32_t kRows = D > 32 ? 32 : kWave;
    alignas(16) float y[kRows][D + 4];  // rows padded to 16 bytes so a lane reads 4 coordinates per access
    float scale[kRows];                 // adjoint weight of the sample (gI_p / N_p)
    uint32_t q[kRows];                  // tile-local pixel of the sample
};

// Writes this lane's part of its sample into row lane % kRows (rows r < count are valid).
template <int D>
__device__ __forceinline__ void stage_rows(StageLds<D>& ST, const float (&x)[kGen<D>], uint32_t count) {
    const uint32_t r = lane_id() % StageLds<D>::kRows;
    const uint32_t j0 = gen_first_dim<D>();
    if (r < count) {
#pragma unroll
        for (int jj = 0; jj < kGen<D>; ++jj) ST.y[r][j0 + jj] = x[jj];
    }
}

// Loads this lane's lobe parameters for group kg: st = kKappa e^-l, b = -c st (zero when the
// lane owns no lobe or the dimension is unused, so those terms vanish).
template <int D>
__device__ __forceinline__ void load_lobe(const Args& a, uint32_t kg, float (&st)[LobeLayout<D>::DH],
                                          float (&b)[LobeLayout<D>::DH], float* w, uint32_t* lobe, bool* own) {
    using LL = LobeLayout<D>;
    const uint32_t lane = lane_id();
    const uint32_t h = lane / LL::LPG;
    const uint32_t k = kg * LL::LPG + lane % LL::LPG;
    *lobe = k;
    *own = k < a.L;
    const uint32_t d = a.d, L = a.L;
    // One base pointer per parameter block, indexed with the unrolled jj: keeps a single 64-bit
    // address live instead of one per dimension.
    const float* pc = a.params + (*own ? uint64_t(k) * d + h * LL::DH : 0);
    const float* pl = pc + uint64_t(L) * d;
#pragma unroll
    for (int jj = 0; jj < LL::DH; ++jj) {
        const uint32_t j = h * LL::DH + jj;
        if (*own && j < d) {
            const float c = pc[jj];
            const float l = pl[jj];
            st[jj] = kKappa * expf(-l);
            b[jj] = -c * st[jj];
        } else {
            st[jj] = 0.0f;
            b[jj] = 0.0f;
        }
    }
    *w = *own ? a.params[2 * L * d + k] : 0.0f;
}

// E = sum_j t_j^2 over all d dimensions of this lane's lobe for staged sample m; t receives
// this lane's half of the t_j.
template <int D>
__device__ __forceinline__ float lobe_exponent(const StageLds<D>& ST, uint32_t m, const float (&st)[LobeLayout<D>::DH],
                                               const float (&b)[LobeLayout<D>::DH], float (&t)[LobeLayout<D>::DH]) {
    using LL = LobeLayout<D>;
    const uint32_t h = lane_id() / LL::LPG;
    const float* y = &ST.y[m][h * LL::DH];
    float e = 0.0f;
#pragma unroll
    for (int jj = 0; jj < LL::DH; ++jj) {
        t[jj] = fmaf(y[jj], st[jj], b[jj]);
        e = fmaf(t[jj], t[jj], e);
    }
    if constexpr (LL::H == 2) {
        // Both halves of the sum in every lane (v_permlane32_swap: no LDS round trip).
        const auto h2 = __builtin_amdgcn_permlane32_swap(__float_as_uint(e), __float_as_uint(e), false, false);
        e = __uint_as_float(h2[0]) + __uint_as_float(h2[1]);
    }
    return e;
}

// ---------------------------------------------------------- lobes forward ----

// Window sums of the tile's pixels into res[q] (one wave_sum per pixel and lobe group).
template <int D, uint32_t SK, bool NUS, bool SHIFT, bool BACK>
__device__ __forceinline__ void lobes_fwd_tile(const Args& a, const SamplerLds<D>& S, PixelLds<D>& PX,
                                               StageLds<D>& ST, float* res, uint32_t task, const TileInfo& ti) {
    using LL = LobeLayout<D>;
    const uint32_t lane = lane_id();
    const uint32_t half = lane / LL::LPG;
    const uint32_t groups = (a.L + LL::LPG - 1) / LL::LPG;
    res[lane] = 0.0f;
    wave_sync();
    for (uint32_t kg = 0; kg < groups; ++kg) {
        float st[LL::DH], b[LL::DH], w;
        uint32_t lobe;
        bool own;
        load_lobe<D>(a, kg, st, b, &w, &lobe, &own);
        if (half != 0) w = 0.0f;  // both halves form G; one adds w G
        float acc = 0.0f;
        uint32_t cur = 0xFFFFFFFFu;
        auto flush = [&]() {
            if (cur != 0xFFFFFFFFu) {
                const float s = wave_sum(acc);
                if (lane == 0) res[cur] += s;
            }
            acc = 0.0f;
        };
        walk_tile<D, SK, NUS, SHIFT, BACK, true>(
            a, S, PX, task, ti.n, ti.inb, ti.off, ti.total, [&](uint32_t) {},
            [&](const float (&x)[kGen<D>], uint32_t count, uint32_t q, uint32_t, bool is_big, uint32_t, uint32_t) {
                stage_rows<D>(ST, x, count);
                if (lane < count) ST.q[lane] = q;
                wave_sync();
                if (is_big) {
                    // The whole round belongs to pixel q: no per-sample bookkeeping, and two
                    // samples per iteration for independent work between the dependent steps.
                    const uint32_t qb = __builtin_amdgcn_readfirstlane(q);
                    if (qb != cur) {
                        flush();
                        cur = qb;
                    }
#pragma unroll 2
                    for (uint32_t m = 0; m < count; ++m) {
                        float t[LL::DH];
                        acc = fmaf(w, exp2_neg(lobe_exponent<D>(ST, m, st, b, t)), acc);
                    }
                } else {
                    for (uint32_t m = 0; m < count; ++m) {
                        const uint32_t qm = __builtin_amdgcn_readfirstlane(ST.q[m]);  // same for all lanes
                        if (qm != cur) {
                            flush();
                            cur = qm;
                        }
                        float t[LL::DH];
                        const float e = lobe_exponent<D>(ST, m, st, b, t);
                        acc = fmaf(w, exp2_neg(e), acc);
                    }
                }
                wave_sync();
            },
            [&](uint32_t) {});
        flush();
        wave_sync();
    }
}

// Up to 32 dimensions compiled for five blocks of four wavefronts per CU (at most 102 registers).
template <int D, uint32_t SK, bool NUS, bool SHIFT, bool BACK>
__global__ __launch_bounds__(kBlock, D > 32 ? 1 : 5) void lobes_fwd(Args a) {
    __shared__ SamplerLds<D> S;
    __shared__ PixelLds<D> PXs[kWavesPerBlock];
    __shared__ StageLds<D> STs[kWavesPerBlock];
    __shared__ float RES[kWavesPerBlock][kTile];
    stage_sampler<D, SK, NUS>(S, a);
    __syncthreads();
    const uint32_t wv = threadIdx.x >> 6;
    for_each_task(a, [&](uint32_t task) {
        const TileInfo ti = tile_info(a, task);
        lobes_fwd_tile<D, SK, NUS, SHIFT, BACK>(a, S, PXs[wv], STs[wv], RES[wv], task, ti);
        if (ti.inb) write_pixel(a, ti.p, RES[wv][lane_id()]);
        wave_sync();
    });
}

// ---------------------------------------------------------- lobes adjoint ----

// Adds sum over the tile's samples of gscale(pixel) * d f / d theta into the accumulator
// (c and l entries still carry the factor kKappa^2 that the final kernel removes).
template <int D, uint32_t SK, bool NUS, bool SHIFT, bool BACK>
__device__ __forceinline__ void lobes_bwd_tile(const Args& a, const SamplerLds<D>& S, PixelLds<D>& PX,
                                               StageLds<D>& ST, uint32_t task, const TileInfo& ti, float gscale) {
    using LL = LobeLayout<D>;
    const uint32_t lane = lane_id();
    const uint32_t half = lane / LL::LPG;
    const uint32_t groups = (a.L + LL::LPG - 1) / LL::LPG;
    for (uint32_t kg = 0; kg < groups; ++kg) {
        float st[LL::DH], b[LL::DH], w;
        uint32_t lobe;
        bool own;
        load_lobe<D>(a, kg, st, b, &w, &lobe, &own);
        float acc_c[LL::DH], acc_l[LL::DH], acc_w = 0.0f;
#pragma unroll
        for (int jj = 0; jj < LL::DH; ++jj) acc_c[jj] = acc_l[jj] = 0.0f;
        walk_tile<D, SK, NUS, SHIFT, BACK, true>(
            a, S, PX, task, ti.n, ti.inb, ti.off, ti.total, [&](uint32_t) {},
            [&](const float (&x)[kGen<D>], uint32_t count, uint32_t q, uint32_t, bool, uint32_t, uint32_t) {
                const float sc = __shfl(gscale, q, kWave);
                stage_rows<D>(ST, x, count);
                if (lane < count) ST.scale[lane] = sc;
                wave_sync();
                {
#pragma unroll 2
                    for (uint32_t m = 0; m < count; ++m) {
                        float t[LL::DH];
                        const float e = lobe_exponent<D>(ST, m, st, b, t);
                        const float aG = ST.scale[m] * exp2_neg(e);
                        acc_w += aG;
                        const float gw = aG * w;
                        if constexpr (D > 32) {
                            // 32 dimensions per lane: t is formed again from the staged sample
                            // rather than kept, which frees 32 registers (two waves per SIMD).
                            const float* y = &ST.y[m][half * LL::DH];
#pragma unroll
                            for (int jj = 0; jj < LL::DH; ++jj) {
                                const float tj = fmaf(y[jj], st[jj], b[jj]);
                                const float gt = gw * tj;
                                acc_c[jj] = add_nc(acc_c[jj], gt);
                                acc_l[jj] = fmaf(gt, tj, acc_l[jj]);
                            }
                        } else {
#pragma unroll
                            for (int jj = 0; jj < LL::DH; ++jj) {
                                const float gt = gw * t[jj];
                                acc_c[jj] = add_nc(acc_c[jj], gt);
                                acc_l[jj] = fmaf(gt, t[jj], acc_l[jj]);
                            }
                        }
                    }
                    wave_sync();
                }
            },
            [&](uint32_t) {});
        if (own) {
            const uint32_t d = a.d, L = a.L;
            uint32_t ec = lobe * d + half * LL::DH;
            asm volatile("" : "+v"(ec));  // formed per task: keeps the entry addresses from being hoisted
#pragma unroll
            for (int jj = 0; jj < LL::DH; ++jj) {
                if (half * LL::DH + jj < d) {
                    acc_add(a, ec + jj, acc_c[jj] * st[jj]);
                    acc_add(a, L * d + ec + jj, acc_l[jj]);
                }
            }
            if (half == 0) acc_add(a, 2 * L * d + lobe, acc_w);
        }
    }
}

template <int D, uint32_t SK, bool NUS, bool SHIFT, bool BACK>
__global__ __launch_bounds__(kBlock) void lobes_bwd(Args a) {
    __shared__ SamplerLds<D> S;
    __shared__ PixelLds<D> PXs[kWavesPerBlock];
    __shared__ StageLds<D> STs[kWavesPerBlock];
    stage_sampler<D, SK, NUS>(S, a);
    __syncthreads();
    const uint32_t wv = threadIdx.x >> 6;
    for_each_task(a, [&](uint32_t task) {
        const TileInfo ti = tile_info(a, task);
        const uint32_t N = ti.inb ? a.counts[ti.p] : 0u;
        const float gscale = (ti.inb && N) ? a.grad_means[ti.p] / static_cast<float>(N) : 0.0f;
        lobes_bwd_tile<D, SK, NUS, SHIFT, BACK>(a, S, PXs[wv], STs[wv], task, ti, gscale);
    });
}

// ------------------------------------------------------ fused L2 training step ----
//
// L = (1/P) sum_p (I_p - T_p)^2: the estimate of each pixel, dL/dI_p = 2 (I_p - T_p) / P and
// the adjoint over the same samples in one kernel.  Accumulator entries: [dL/dtheta, loss sum].
// The adjoint's per-pixel sums  sum_i G,  sum_i w G t_j  and  sum_i w G t_j^2  do not depend on
// dL/dI_p, only their final scaling does.  When all lobes fit one lane group (SINGLE), a big
// pixel's samples are generated once and feed the estimate and these sums together; packed
// pixels, whose samples share rounds, get their estimates from a forward walk first.  With more
// lobes than one group the estimate needs every group first, and for d > 8 a lane has no
// registers left for the unscaled sums, so such launches (SINGLE = false) run the forward walk
// and then the adjoint walk.  Up to 32 dimensions the kernel is compiled for four blocks of four
// wavefronts per CU (at most 128 registers; 37 KB of LDS per block): at 1920x1080 x 64 spp,
// d = 8, it took 9.0-9.7 ms against 9.4-10.3 ms with 129 registers (three wavefronts per SIMD).
template <int D, uint32_t SK, bool NUS, bool SHIFT, bool BACK, bool SINGLE>
__global__ __launch_bounds__(kBlock, D > 32 ? 1 : 4) void lobes_step(Args a) {
    using LL = LobeLayout<D>;
    __shared__ SamplerLds<D> S;
    __shared__ PixelLds<D> PXs[kWavesPerBlock];
    __shared__ StageLds<D> STs[kWavesPerBlock];
    __shared__ float RES[kWavesPerBlock][kTile];
    stage_sampler<D, SK, NUS>(S, a);
    __syncthreads();
    const uint32_t wv = threadIdx.x >> 6;
    PixelLds<D>& PX = PXs[wv];
    StageLds<D>& ST = STs[wv];
    const uint32_t lane = lane_id();
    const uint32_t half = lane / LL::LPG;
    const float invP = 1.0f / static_cast<float>(a.num_pixels);
    for_each_task(a, [&](uint32_t task) {
        const TileInfo ti = tile_info(a, task);
        if constexpr (SINGLE) {
            // (1) Packed pixels (fewer than 64 samples): forward sums first, so that their
            // samples carry a known scale dL/dI_p / N_p through the adjoint walk below.
            TileInfo ts = ti;
            ts.n = ti.ns;  // hides the big pixels from this walk
            lobes_fwd_tile<D, SK, NUS, SHIFT, BACK>(a, S, PX, ST, RES[wv], task, ts);
            const uint32_t N = ti.inb ? a.counts[ti.p] : 0u;
            float gs = 0.0f, sq = 0.0f;
            if (ti.inb && ti.n < kWave) {  // packed or empty pixel
                const float I = N ? RES[wv][lane] / static_cast<float>(N) : 0.0f;
                const float diff = I - a.target[ti.p];
                if (a.means) a.means[ti.p] = I;
                sq = diff * diff;
                gs = N ? 2.0f * diff * invP / static_cast<float>(N) : 0.0f;
            }
            float loss = wave_sum(sq);
            wave_sync();
            // (2) One walk over every sample.  A big pixel's rounds hold only its own samples:
            // its estimate and the unscaled adjoint sums  sum_i G,  sum_i w G t_j,
            // sum_i w G t_j^2  accumulate together, and at the end of the pixel the sums are
            // scaled by dL/dI_p / N_p into the lobe's totals.  Packed samples enter the same
            // sums already scaled.  No pixel bookkeeping runs inside the per-sample loop.
            float st[LL::DH], b[LL::DH], w;
            uint32_t lobe;
            bool own;
            load_lobe<D>(a, 0, st, b, &w, &lobe, &own);
            const float wf = half == 0 ? w : 0.0f;  // both halves form G; one adds it to the estimate
            // The lobe's running totals live in LDS (touched once per pixel).
            __shared__ float ACC[kWavesPerBlock][2 * LL::DH + 1][kWave];
            float(&acc)[2 * LL::DH + 1][kWave] = ACC[wv];
#pragma unroll
            for (int k = 0; k < 2 * LL::DH + 1; ++k) acc[k][lane] = 0.0f;
            float pf = 0.0f, pw = 0.0f, pc[LL::DH], pl[LL::DH];
#pragma unroll
            for (int jj = 0; jj < LL::DH; ++jj) pc[jj] = pl[jj] = 0.0f;
            auto add_sums = [&](float scale) {
                acc[2 * LL::DH][lane] = fmaf(scale, pw, acc[2 * LL::DH][lane]);
#pragma unroll
                for (int jj = 0; jj < LL::DH; ++jj) {
                    acc[jj][lane] = fmaf(scale, pc[jj], acc[jj][lane]);
                    acc[LL::DH + jj][lane] = fmaf(scale, pl[jj], acc[LL::DH + jj][lane]);
                }
                pf = pw = 0.0f;
#pragma unroll
                for (int jj = 0; jj < LL::DH; ++jj) pc[jj] = pl[jj] = 0.0f;
            };
            walk_tile<D, SK, NUS, SHIFT, BACK, true>(
                a, S, PX, task, ti.n, ti.inb, ti.off, ti.total, [&](uint32_t) {},
                [&](const float (&x)[kGen<D>], uint32_t count, uint32_t q, uint32_t, bool is_big, uint32_t, uint32_t) {
                    const float sc = is_big ? 1.0f : __shfl(gs, q, kWave);
                    stage_rows<D>(ST, x, count);
                    if (lane < count) ST.scale[lane] = sc;
                    wave_sync();
                    {
#pragma unroll 2
                        for (uint32_t m = 0; m < count; ++m) {
                            float t[LL::DH];
                            const float G = exp2_neg(lobe_exponent<D>(ST, m, st, b, t));
                            const float g = ST.scale[m] * G;
                            pf = fmaf(wf, G, pf);
                            pw += g;
                            const float wg = w * g;
#pragma unroll
                            for (int jj = 0; jj < LL::DH; ++jj) {
                                const float gt = wg * t[jj];
                                pc[jj] = add_nc(pc[jj], gt);
                                pl[jj] = fmaf(gt, t[jj], pl[jj]);
                            }
                        }
                        wave_sync();
                    }
                },
                [&](uint32_t q) {
                    const uint32_t pp = task * kTile + q;
                    const uint32_t Nq = a.counts[pp];  // >= 64
                    const float I = wave_sum(pf) / static_cast<float>(Nq);
                    const float diff = I - a.target[pp];
                    if (lane == 0 && a.means) a.means[pp] = I;
                    loss = fmaf(diff, diff, loss);
                    add_sums(2.0f * diff * invP / static_cast<float>(Nq));
                });
            add_sums(1.0f);  // packed samples: already scaled
            if (own) {
                const uint32_t d = a.d, L = a.L;
                uint32_t ec = lobe * d + half * LL::DH;
                asm volatile("" : "+v"(ec));  // formed per task: keeps the entry addresses from being hoisted
#pragma unroll
                for (int jj = 0; jj < LL::DH; ++jj) {
                    if (half * LL::DH + jj < d) {
                        acc_add(a, ec + jj, acc[jj][lane] * st[jj]);
                        acc_add(a, L * d + ec + jj, acc[LL::DH + jj][lane]);
                    }
                }
                if (half == 0) acc_add(a, 2 * L * d + lobe, acc[2 * LL::DH][lane]);
            }
            if (lane == 0) acc_add(a, a.n_theta, loss);
            wave_sync();
        } else {
            // forward walk over every lobe group, per-pixel loss gradient, adjoint walk
            lobes_fwd_tile<D, SK, NUS, SHIFT, BACK>(a, S, PX, ST, RES[wv], task, ti);
            const uint32_t N = ti.inb ? a.counts[ti.p] : 0u;
            float gscale = 0.0f, sq = 0.0f;
            if (ti.inb) {
                const float I = N ? RES[wv][lane] / static_cast<float>(N) : 0.0f;
                const float diff = I - a.target[ti.p];
                if (a.means) a.means[ti.p] = I;
                sq = diff * diff;
                gscale = N ? 2.0f * diff * invP / static_cast<float>(N) : 0.0f;
            }
            const float loss = wave_sum(sq);
            wave_sync();
            lobes_bwd_tile<D, SK, NUS, SHIFT, BACK>(a, S, PX, ST, task, ti, gscale);
            if (lane == 0) acc_add(a, a.n_theta, loss);
        }
    });
}

// Clears n words (a kernel rather than a memset, so that graph captures replay it correctly).
__global__ __launch_bounds__(256) void zero_words(unsigned long long* __restrict__ w, uint64_t n) {
    for (uint64_t i = blockIdx.x * uint64_t(256) + threadIdx.x; i < n; i += uint64_t(gridDim.x) * 256) w[i] = 0ull;
}

// Final step of the exact accumulation: entry e = sum of its digits over the copies (int64, exact),
// carries propagated so that digits 0..7 lie in [0, 2^32) and the top one holds the sign, then
// value = sum_k digit_k 2^(32k - 149), formed from the top digit down in FP64.  grad[e] += value
// times the entry's scale (1/kKappa^2 for centres and log-widths); the loss entry (e = n_theta,
// L2 step) adds value / P to *loss.  A non-finite addend makes the entry NaN.
__global__ __launch_bounds__(256) void acc_finalize(const unsigned long long* __restrict__ acc, uint32_t n_row,
                                                    uint32_t n_theta, uint32_t LD, float* __restrict__ grad,
                                                    float* __restrict__ loss, uint32_t num_pixels) {
    const uint32_t e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n_row) return;
    long long dg[kAccWords];
#pragma unroll
    for (uint32_t k = 0; k < kAccWords; ++k) dg[k] = 0;
    for (uint32_t c = 0; c < kAccCopies; ++c) {
        const unsigned long long* w = acc + (uint64_t(c) * n_row + e) * kAccWords;
#pragma unroll
        for (uint32_t k = 0; k < kAccWords; ++k) dg[k] += static_cast<long long>(w[k]);
    }
#pragma unroll
    for (uint32_t k = 0; k + 1 < kAccDigits; ++k) {
        const long long carry = dg[k] >> 32;  // floor division by 2^32
        dg[k] -= carry * 4294967296ll;
        dg[k + 1] += carry;
    }
    double v = static_cast<double>(dg[kAccDigits - 1]);
    for (int k = static_cast<int>(kAccDigits) - 2; k >= 0; --k) v = v * 4294967296.0 + static_cast<double>(dg[k]);
    v = ldexp(v, -149);
    if (dg[kAccWords - 1] != 0) v = __builtin_nan("");
    if (e < n_theta) {
        const double scale = e < 2 * LD ? 1.0 / (static_cast<double>(kKappa) * kKappa) : 1.0;
        grad[e] += static_cast<float>(v * scale);
    } else if (loss) {
        *loss += static_cast<float>(v / num_pixels);
    }
}

__global__ void reset_queue(uint32_t* q) {
    if (threadIdx.x < kQueues) q[threadIdx.x * kQueueStride] = 0u;
}

// ------------------------------------------------ materialised samples (plain) ----

template <int D, uint32_t SK, bool NUS, bool SHIFT, bool BACK>
__global__ __launch_bounds__(kBlock) void pixel_samples(Args a) {
    __shared__ SamplerLds<D> S;
    __shared__ PixelLds<D> PXs[kWavesPerBlock];
    // per-pixel seeds of packed pixels in LDS (small dimension counts only)
    constexpr bool kPacked = D <= 8;
    __shared__ PackedSeeds<kPacked ? D : 1> PKs[kPacked ? kWavesPerBlock : 1];
    stage_sampler<D, SK, NUS>(S, a);
    __syncthreads();
    PixelLds<D>& PX = PXs[threadIdx.x >> 6];
    PackedSeeds<D>* PK = nullptr;
    if constexpr (kPacked) {
        if (NUS || SHIFT || SK == QMC_SAMPLER_LATTICE) PK = &PKs[threadIdx.x >> 6];
    }
    const uint32_t lane = lane_id();
    for_each_task(a, [&](uint32_t task) {
        const TileInfo ti = tile_info(a, task);
        walk_tile<D, SK, NUS, SHIFT, BACK, false>(
            a, S, PX, task, ti.n, ti.inb, ti.off, ti.total, [&](uint32_t) {},
            [&](const float (&x)[kGen<D>], uint32_t count, uint32_t, uint32_t pp, bool, uint32_t, uint32_t i) {
                if (lane % kRoundSamples<D> < count) {
                    const uint64_t off = a.offsets[pp] + i;
                    const uint32_t j0 = gen_first_dim<D>();
#pragma unroll
                    for (int jj = 0; jj < kGen<D>; ++jj)
                        if (j0 + jj < a.d) a.out[uint64_t(j0 + jj) * a.out_ld + off] = x[jj];
                }
            },
            [&](uint32_t) {}, PK);
    });
}

// Exclusive scan of counts into u64 offsets: per-block scans of 1024 counts, a scan of the
// block totals, then the block prefixes are added.
__global__ __launch_bounds__(256) void scan_blocks(const uint32_t* __restrict__ counts, uint32_t n,
                                                   uint64_t* __restrict__ offsets, uint64_t* __restrict__ block_tot) {
    __shared__ uint64_t part[256];
    const uint32_t base = blockIdx.x * 1024 + threadIdx.x * 4;
    uint64_t v[4], run = 0;
    for (int r = 0; r < 4; ++r) {
        v[r] = base + r < n ? counts[base + r] : 0u;
        run += v[r];
    }
    part[threadIdx.x] = run;
    __syncthreads();
    for (uint32_t o = 1; o < 256; o <<= 1) {
        const uint64_t add = threadIdx.x >= o ? part[threadIdx.x - o] : 0;
        __syncthreads();
        part[threadIdx.x] += add;
        __syncthreads();
    }
    uint64_t ex = part[threadIdx.x] - run;
    for (int r = 0; r < 4; ++r) {
        if (base + r < n) offsets[base + r] = ex;
        ex += v[r];
    }
    if (threadIdx.x == 255) block_tot[blockIdx.x] = part[255];
}

__global__ void scan_totals(uint64_t* __restrict__ block_tot, uint32_t nblocks, uint64_t* __restrict__ offsets,
                            uint32_t n) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    uint64_t run = 0;
    for (uint32_t b = 0; b < nblocks; ++b) {
        const uint64_t t = block_tot[b];
        block_tot[b] = run;
        run += t;
    }
    offsets[n] = run;
}

__global__ __launch_bounds__(256) void scan_add(uint64_t* __restrict__ offsets, uint32_t n,
                                                const uint64_t* __restrict__ block_tot) {
    const uint32_t e = blockIdx.x * 256 + threadIdx.x;
    if (e < n) offsets[e] += block_tot[e / 1024];
}

// -------------------------------------------------------------------- host ----

// Workspace: the task queues (kQueueBytes), then for the adjoint the exact accumulator, or for the
// Genz forward pass the Sobol' tables (4 KB), the bucket sizes (512 bytes), the per-wavefront
// counts and the pixel list.
struct Plan {
    size_t queue_off = 0, acc_off = kQueueBytes, tab_off = kQueueBytes, total_off = kQueueBytes + 4096,
           wave_off = kQueueBytes + 4096 + 512, list_off = 0, total = kQueueBytes;
    uint32_t num_tasks = 0, n_theta = 0, n_row = 0, bucket_waves = 0;
    uint64_t acc_words = 0;
};

// mode: 0 forward, 1 adjoint, 2 fused L2 step (partial rows carry one extra loss entry).
Plan make_plan(const qmc_integrand* ig, uint32_t P, int mode) {
    Plan pl;
    pl.num_tasks = (P + kTile - 1) / kTile;
    if (ig && ig->kind == QMC_F_LOBES) pl.n_theta = ig->num_lobes * (2 * ig->d + 1);
    pl.n_row = pl.n_theta + (mode == 2 ? 1u : 0u);
    if (mode != 0) {
        pl.acc_words = uint64_t(kAccCopies) * pl.n_row * kAccWords;
        pl.total = pl.acc_off + pl.acc_words * 8;
    } else if (ig && ig->kind == QMC_F_GENZ) {
        auto up = [](size_t x) { return (x + 255) & ~size_t(255); };
        pl.bucket_waves = static_cast<uint32_t>((uint64_t(P) + kBucketPixels - 1) / kBucketPixels);
        pl.list_off = pl.wave_off + up(size_t(kBuckets) * pl.bucket_waves * 4);
        pl.total = pl.list_off + up(size_t(P) * 4);
    }
    return pl;
}

qmc_status validate_sampler(const char* who, const qmc_sampler* sp, uint32_t d) {
    if (sp->kind < QMC_SAMPLER_SOBOL || sp->kind > QMC_SAMPLER_XOR_TABLE)
        return fail(QMC_ERR_INVALID_ARGUMENT, "%s: unknown sampler kind %u", who, sp->kind);
    if (sp->kind == QMC_SAMPLER_XOR_TABLE) {
        if (sp->flags) return fail(QMC_ERR_INVALID_ARGUMENT, "%s: the XOR table sampler takes no flags", who);
        if (!sp->xor_scramble || !sp->xor_reorder)
            return fail(QMC_ERR_INVALID_ARGUMENT, "%s: XOR table sampler needs its scramble and reorder tables", who);
        const uint64_t n = sp->points_ld;
        if (n == 0 || n > (uint64_t(1) << 32) || (n & (n - 1)))
            return fail(QMC_ERR_INVALID_ARGUMENT, "%s: XOR table sampler needs 2^k stored points, k <= 32", who);
    }
    if (!sp->table) return fail(QMC_ERR_INVALID_ARGUMENT, "%s: sampler table is NULL", who);
    if (sp->s == 0 || sp->s > QMC_MAX_DIMS) return fail(QMC_ERR_OUT_OF_RANGE, "%s: sampler s out of range", who);
    const uint32_t lattice_only = QMC_PIXEL_RANDOM_GENERATOR | QMC_LATTICE_INSTANCES4 | QMC_PIXEL_HILBERT_SHIFT;
    const uint32_t allowed =
        QMC_PIXEL_NUS | QMC_PIXEL_SHIFT | QMC_SHIFT_XOR | QMC_LATTICE_BACKWARD | QMC_PIXEL_TABLE_SHIFT | lattice_only;
    if (sp->flags & ~allowed) return fail(QMC_ERR_INVALID_ARGUMENT, "%s: unknown sampler flags", who);
    if (sp->kind != QMC_SAMPLER_SOBOL && (sp->flags & QMC_PIXEL_NUS))
        return fail(QMC_ERR_INVALID_ARGUMENT, "%s: only the Sobol' sampler has a nested scramble", who);
    if (sp->kind != QMC_SAMPLER_LATTICE && (sp->flags & lattice_only))
        return fail(QMC_ERR_INVALID_ARGUMENT, "%s: generator and Hilbert-shift options are for the lattice sampler",
                    who);
    if ((sp->flags & QMC_PIXEL_TABLE_SHIFT) && (!(sp->flags & QMC_PIXEL_SHIFT) || !sp->shift_table))
        return fail(QMC_ERR_INVALID_ARGUMENT, "%s: table rotations need QMC_PIXEL_SHIFT and a shift table", who);
    if ((sp->flags & QMC_LATTICE_INSTANCES4) && !(sp->flags & QMC_PIXEL_RANDOM_GENERATOR))
        return fail(QMC_ERR_INVALID_ARGUMENT, "%s: four instances need per-pixel random generators", who);
    if (sp->kind == QMC_SAMPLER_POINTS && !sp->offsets)
        return fail(QMC_ERR_INVALID_ARGUMENT, "%s: POINTS sampler needs offsets", who);
    if (d > sp->s) return fail(QMC_ERR_INVALID_ARGUMENT, "%s: integrand needs d = %u > sampler s = %u", who, d, sp->s);
    return QMC_OK;
}

// The Hilbert shift indexes the 2^k x 2^k square covering the image; k <= 15 keeps the curve
// index and the exact base-3 inversion within 64-bit arithmetic.
qmc_status validate_hilbert(const char* who, const qmc_sampler* sp, uint32_t W, uint32_t H) {
    if ((sp->flags & QMC_PIXEL_HILBERT_SHIFT) && std::max(W, H) > 32768u)
        return fail(QMC_ERR_OUT_OF_RANGE, "%s: the Hilbert shift supports images up to 32768 pixels wide and high",
                    who);
    return QMC_OK;
}

qmc_status validate(const char* who, qmc_context ctx, const qmc_sampler* sp, const qmc_integrand* ig, uint32_t W,
                    uint32_t H, const uint32_t* counts, uint32_t begin, uint32_t end, bool backward) {
    if (!ctx || !sp || !ig) return fail(QMC_ERR_INVALID_ARGUMENT, "%s: NULL context, sampler or integrand", who);
    if (ig->kind == QMC_F_GENZ) {
        if (ig->d != 8) return fail(QMC_ERR_UNSUPPORTED, "%s: the Genz integrand has d = 8", who);
        if (!ig->pixel_params) return fail(QMC_ERR_INVALID_ARGUMENT, "%s: Genz pixel_params is NULL", who);
        if (backward) return fail(QMC_ERR_UNSUPPORTED, "%s: the adjoint exists for the lobe integrand only", who);
    } else if (ig->kind == QMC_F_LOBES) {
        if (ig->d == 0 || ig->d > QMC_MAX_DIMS) return fail(QMC_ERR_OUT_OF_RANGE, "%s: lobe dimension out of range", who);
        if (ig->num_lobes == 0 || ig->num_lobes > 65536)
            return fail(QMC_ERR_OUT_OF_RANGE, "%s: num_lobes out of range", who);
        if (!ig->params) return fail(QMC_ERR_INVALID_ARGUMENT, "%s: lobe params is NULL", who);
    } else {
        return fail(QMC_ERR_INVALID_ARGUMENT, "%s: unknown integrand kind %u", who, ig->kind);
    }
    qmc_status st = validate_sampler(who, sp, ig->d);
    if (st == QMC_OK) st = validate_hilbert(who, sp, W, H);
    if (st != QMC_OK) return st;
    if (uint64_t(W) * H == 0 || uint64_t(W) * H > 0xFFFFFFFFull - kTile)
        return fail(QMC_ERR_OUT_OF_RANGE, "%s: image size out of range", who);
    if (!counts) return fail(QMC_ERR_INVALID_ARGUMENT, "%s: counts is NULL", who);
    if (begin > end) return fail(QMC_ERR_INVALID_ARGUMENT, "%s: sample_begin > sample_end", who);
    return QMC_OK;
}

// Launches Fam::go<SK, NUS, SHIFT, BACK> for the sampler's kind and flags; only the
// meaningful combinations are instantiated (scrambling for Sobol' only, backward order for
// the lattice only, materialised points and the XOR table sampler without either).
template <typename Fam>
void dispatch_sampler(uint32_t skind, bool nus, bool shift, bool back, uint32_t grid, hipStream_t hs, const Args& a) {
    if (skind == QMC_SAMPLER_SOBOL) {
        if (nus) {
            if (shift) Fam::template go<QMC_SAMPLER_SOBOL, true, true, false>(grid, hs, a);
            else Fam::template go<QMC_SAMPLER_SOBOL, true, false, false>(grid, hs, a);
        } else {
            if (shift) Fam::template go<QMC_SAMPLER_SOBOL, false, true, false>(grid, hs, a);
            else Fam::template go<QMC_SAMPLER_SOBOL, false, false, false>(grid, hs, a);
        }
    } else if (skind == QMC_SAMPLER_LATTICE) {
        if (back) {
            if (shift) Fam::template go<QMC_SAMPLER_LATTICE, false, true, true>(grid, hs, a);
            else Fam::template go<QMC_SAMPLER_LATTICE, false, false, true>(grid, hs, a);
        } else {
            if (shift) Fam::template go<QMC_SAMPLER_LATTICE, false, true, false>(grid, hs, a);
            else Fam::template go<QMC_SAMPLER_LATTICE, false, false, false>(grid, hs, a);
        }
    } else if (skind == QMC_SAMPLER_XOR_TABLE) {
        Fam::template go<QMC_SAMPLER_XOR_TABLE, false, false, false>(grid, hs, a);
    } else if constexpr (Fam::kPoints) {
        Fam::template go<QMC_SAMPLER_POINTS, false, false, false>(grid, hs, a);
    }
}

struct GenzFam {
    static constexpr bool kPoints = true;
    template <uint32_t SK, bool NUS, bool SH, bool BK>
    static void go(uint32_t grid, hipStream_t hs, const Args& a) {
        hipLaunchKernelGGL((genz_fwd<SK, NUS, SH, BK>), dim3(grid), dim3(kBlock), 0, hs, a);
    }
};

template <int D>
struct LobesFwdFam {
    static constexpr bool kPoints = true;
    template <uint32_t SK, bool NUS, bool SH, bool BK>
    static void go(uint32_t grid, hipStream_t hs, const Args& a) {
        hipLaunchKernelGGL((lobes_fwd<D, SK, NUS, SH, BK>), dim3(grid), dim3(kBlock), 0, hs, a);
    }
};

template <int D>
struct LobesBwdFam {
    static constexpr bool kPoints = true;
    template <uint32_t SK, bool NUS, bool SH, bool BK>
    static void go(uint32_t grid, hipStream_t hs, const Args& a) {
        hipLaunchKernelGGL((lobes_bwd<D, SK, NUS, SH, BK>), dim3(grid), dim3(kBlock), 0, hs, a);
    }
};

template <int D, bool SINGLE>
struct LobesStepFam {
    static constexpr bool kPoints = true;
    template <uint32_t SK, bool NUS, bool SH, bool BK>
    static void go(uint32_t grid, hipStream_t hs, const Args& a) {
        hipLaunchKernelGGL((lobes_step<D, SK, NUS, SH, BK, SINGLE>), dim3(grid), dim3(kBlock), 0, hs, a);
    }
};

template <int D>
struct SamplesFam {
    static constexpr bool kPoints = false;
    template <uint32_t SK, bool NUS, bool SH, bool BK>
    static void go(uint32_t grid, hipStream_t hs, const Args& a) {
        hipLaunchKernelGGL((pixel_samples<D, SK, NUS, SH, BK>), dim3(grid), dim3(kBlock), 0, hs, a);
    }
};

uint32_t hilbert_order_of(uint32_t W, uint32_t H) {
    uint32_t k = 1;
    while ((uint64_t(1) << k) < std::max(W, H)) ++k;
    return k;
}

Args base_args(const qmc_sampler* sp, uint32_t d, uint32_t W, uint32_t H, const uint32_t* counts, uint32_t begin,
               uint32_t end) {
    const uint32_t P = W * H;
    Args a{};
    a.lrgen = (sp->flags & QMC_PIXEL_RANDOM_GENERATOR) ? 1u : 0u;
    a.linst4 = (sp->flags & QMC_LATTICE_INSTANCES4) ? 1u : 0u;
    a.lhilbert = (sp->flags & QMC_PIXEL_HILBERT_SHIFT) ? 1u : 0u;
    a.width = W;
    a.hilbert_order = hilbert_order_of(W, H);
    a.skind = sp->kind;
    a.s = sp->s;
    a.seed = sp->seed;
    a.sflags = sp->flags;
    a.sxor = (sp->flags & QMC_SHIFT_XOR) ? 1u : 0u;
    a.table = static_cast<const uint32_t*>(sp->table);
    a.points = static_cast<const float*>(sp->table);
    a.points_ld = sp->points_ld;
    a.offsets = sp->offsets;
    a.xor_scramble = sp->xor_scramble;
    a.xor_reorder = sp->xor_reorder;
    a.xor_mask = static_cast<uint32_t>(sp->points_ld - 1);
    a.shift_table = (sp->flags & QMC_PIXEL_TABLE_SHIFT) ? sp->shift_table : nullptr;
    a.d = d;
    a.num_pixels = P;
    a.counts = counts;
    a.begin = begin;
    a.end = end;
    a.aligned = (begin % kWave) == 0 ? 1u : 0u;
    a.num_tasks = (P + kTile - 1) / kTile;
    return a;
}

uint32_t persistent_grid(const qmc_context ctx, const IntegrateTune& tn, uint32_t num_tasks, Args* a) {
    const uint32_t waves_wanted = std::max<uint32_t>(1, uint32_t(ctx->num_cus) * tn.waves_per_cu);
    const uint32_t task_waves = ((num_tasks + kWavesPerBlock - 1) / kWavesPerBlock) * kWavesPerBlock;
    const uint32_t waves = std::min<uint32_t>(waves_wanted, std::max<uint32_t>(task_waves, kWavesPerBlock));
    const uint32_t grid = (waves + kWavesPerBlock - 1) / kWavesPerBlock;
    a->total_waves = grid * kWavesPerBlock;
    a->dynamic = tn.dynamic;
    return grid;
}

// mode 0: forward; 1: adjoint; 2: fused L2 step (grad_means is the target, sums the loss).
qmc_status integrate_common(const char* who, qmc_context ctx, qmc_stream stream, const qmc_sampler* sp,
                            const qmc_integrand* ig, uint32_t W, uint32_t H, const uint32_t* counts, uint32_t begin,
                            uint32_t end, float* sums, float* means, const float* grad_means, float* grad_params,
                            void* ws, size_t ws_bytes, int mode) {
    const bool backward = mode != 0;
    qmc_status st = validate(who, ctx, sp, ig, W, H, counts, begin, end, backward);
    if (st != QMC_OK) return st;
    if (mode == 0 && !sums && !means) return fail(QMC_ERR_INVALID_ARGUMENT, "%s: sums and means are both NULL", who);
    if (backward && (!grad_means || !grad_params))
        return fail(QMC_ERR_INVALID_ARGUMENT, "%s: %s and grad_params are required", who,
                    mode == 2 ? "target" : "grad_means");
    const uint32_t P = W * H;
    const Plan pl = make_plan(ig, P, mode);
    if (!ws || ws_bytes < pl.total)
        return fail(QMC_ERR_WORKSPACE, "%s: workspace of %zu bytes needed, %zu given", who, pl.total, ws_bytes);
    DeviceGuard guard(ctx->device);
    if (guard.status != QMC_OK) return guard.status;
    hipStream_t hs = as_stream(stream);
    Args a = base_args(sp, ig->d, W, H, counts, begin, end);
    a.fkind = ig->kind;
    a.L = ig->num_lobes;
    a.pixel_seed = ig->pixel_seed;
    a.params = ig->params;
    a.pixel_params = ig->pixel_params;
    a.sums = mode == 2 ? nullptr : sums;
    a.means = means;
    a.grad_means = mode == 2 ? nullptr : grad_means;
    a.target = mode == 2 ? grad_means : nullptr;
    a.queue = reinterpret_cast<uint32_t*>(static_cast<char*>(ws) + pl.queue_off);
    a.acc = reinterpret_cast<unsigned long long*>(static_cast<char*>(ws) + pl.acc_off);
    a.n_theta = pl.n_theta;
    a.n_row = pl.n_row;
    a.bucket_total = reinterpret_cast<uint32_t*>(static_cast<char*>(ws) + pl.total_off);
    a.bucket_wave = reinterpret_cast<uint32_t*>(static_cast<char*>(ws) + pl.wave_off);
    a.bucket_list = reinterpret_cast<uint32_t*>(static_cast<char*>(ws) + pl.list_off);
    a.genz_tab = reinterpret_cast<uint32_t*>(static_cast<char*>(ws) + pl.tab_off);
    a.bucket_waves = pl.bucket_waves;
    const bool genz = !backward && ig->kind == QMC_F_GENZ;
    // the Genz pass runs a task per 64 pixels of a bucket (at most tiles + buckets tasks)
    const uint32_t grid = persistent_grid(ctx, integrate_tune(ctx, ig->kind, ig->d, backward),
                                          genz ? 2 * pl.num_tasks : pl.num_tasks, &a);
    const bool nus = (sp->flags & QMC_PIXEL_NUS) != 0, shift = (sp->flags & QMC_PIXEL_SHIFT) != 0;
    const bool back = (sp->flags & QMC_LATTICE_BACKWARD) != 0;
    clear_launch_error();
    if (a.dynamic) hipLaunchKernelGGL(reset_queue, dim3(1), dim3(kWave), 0, hs, a.queue);
    if (backward) {
        const uint32_t zb = static_cast<uint32_t>(std::min<uint64_t>((pl.acc_words + 255) / 256, 1024));
        hipLaunchKernelGGL(zero_words, dim3(zb), dim3(256), 0, hs, a.acc, pl.acc_words);
    }
    if (genz) {
        const uint32_t bblocks = (pl.bucket_waves + kWavesPerBlock - 1) / kWavesPerBlock;
        hipLaunchKernelGGL(genz_bucket_count, dim3(bblocks), dim3(256), 0, hs, a);
        hipLaunchKernelGGL(genz_bucket_scan, dim3(kBuckets), dim3(1024), 0, hs, a);
        hipLaunchKernelGGL(genz_bucket_fill, dim3(bblocks), dim3(256), 0, hs, a);
    }
    if (!backward) {
        if (ig->kind == QMC_F_GENZ)
            dispatch_sampler<GenzFam>(sp->kind, nus, shift, back, grid, hs, a);
        else if (ig->d <= 8)
            dispatch_sampler<LobesFwdFam<8>>(sp->kind, nus, shift, back, grid, hs, a);
        else
            dispatch_sampler<LobesFwdFam<64>>(sp->kind, nus, shift, back, grid, hs, a);
    } else {
        if (mode == 1) {
            if (ig->d <= 8)
                dispatch_sampler<LobesBwdFam<8>>(sp->kind, nus, shift, back, grid, hs, a);
            else
                dispatch_sampler<LobesBwdFam<64>>(sp->kind, nus, shift, back, grid, hs, a);
        } else if (ig->d <= 8) {
            if (ig->num_lobes <= LobeLayout<8>::LPG)
                dispatch_sampler<LobesStepFam<8, true>>(sp->kind, nus, shift, back, grid, hs, a);
            else
                dispatch_sampler<LobesStepFam<8, false>>(sp->kind, nus, shift, back, grid, hs, a);
        } else {
            // d > 8: a lane's share of the adjoint state (32 dimensions) leaves no registers for
            // a pixel's unscaled sums, so the step runs the forward walk, then the adjoint walk.
            dispatch_sampler<LobesStepFam<64, false>>(sp->kind, nus, shift, back, grid, hs, a);
        }
        hipLaunchKernelGGL(acc_finalize, dim3((pl.n_row + 255) / 256), dim3(256), 0, hs, a.acc, pl.n_row, pl.n_theta,
                           ig->num_lobes * ig->d, grad_params, mode == 2 ? sums : nullptr, P);
    }
    return check_launch(who);
}

}  // namespace
}  // namespace qmc

// Static scratch of qmc_integrate_pixels_l2_step_noalloc (work counter and exact accumulator):
// every device the library runs on holds its own copy until the process ends.  Host code uses
// the address that static_scratch_address() looked up on the device, never this name.
static __device__ __align__(256) unsigned char scratch[QMC_STATIC_SCRATCH_BYTES];

namespace qmc {

qmc_status static_scratch_address(int device, void** ptr) {
    static std::mutex mu;
    static std::map<int, void*> addresses;
    std::lock_guard<std::mutex> lock(mu);
    const auto it = addresses.find(device);
    if (it != addresses.end()) {
        *ptr = it->second;
        return QMC_OK;
    }
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
        return fail(QMC_ERR_DEVICE, "qmc_create: no address for the static scratch on device %d: %s", device,
                    hipGetErrorString(e));
    addresses[device] = p;
    *ptr = p;
    return QMC_OK;
}

}  // namespace qmc

using namespace qmc;

extern "C" qmc_status qmc_workspace_size(qmc_context ctx, const qmc_sampler* sampler, const qmc_integrand* integrand,
                                         uint32_t width, uint32_t height, int backward, size_t* bytes) {
    if (!ctx || !sampler || !integrand || !bytes)
        return fail(QMC_ERR_INVALID_ARGUMENT, "qmc_workspace_size: NULL argument");
    if (backward < 0 || backward > 2) return fail(QMC_ERR_INVALID_ARGUMENT, "qmc_workspace_size: mode must be 0, 1 or 2");
    *bytes = make_plan(integrand, width * height, backward).total;
    return QMC_OK;
}

extern "C" qmc_status qmc_integrate_pixels(qmc_context ctx, qmc_stream stream, const qmc_sampler* sampler,
                                           const qmc_integrand* integrand, uint32_t width, uint32_t height,
                                           const uint32_t* counts, uint32_t sample_begin, uint32_t sample_end,
                                           float* sums, float* means, void* workspace, size_t workspace_bytes) {
    return integrate_common("qmc_integrate_pixels", ctx, stream, sampler, integrand, width, height, counts,
                            sample_begin, sample_end, sums, means, nullptr, nullptr, workspace, workspace_bytes, 0);
}

extern "C" qmc_status qmc_integrate_pixels_backward(qmc_context ctx, qmc_stream stream, const qmc_sampler* sampler,
                                                    const qmc_integrand* integrand, uint32_t width, uint32_t height,
                                                    const uint32_t* counts, uint32_t sample_begin,
                                                    uint32_t sample_end, const float* grad_means, float* grad_params,
                                                    void* workspace, size_t workspace_bytes) {
    return integrate_common("qmc_integrate_pixels_backward", ctx, stream, sampler, integrand, width, height, counts,
                            sample_begin, sample_end, nullptr, nullptr, grad_means, grad_params, workspace,
                            workspace_bytes, 1);
}

extern "C" qmc_status qmc_integrate_pixels_l2_step(qmc_context ctx, qmc_stream stream, const qmc_sampler* sampler,
                                                   const qmc_integrand* integrand, uint32_t width, uint32_t height,
                                                   const uint32_t* counts, const float* target, float* means,
                                                   float* loss, float* grad_params, void* workspace,
                                                   size_t workspace_bytes) {
    const char* who = "qmc_integrate_pixels_l2_step";
    if (!loss) return fail(QMC_ERR_INVALID_ARGUMENT, "%s: loss is NULL", who);
    return integrate_common(who, ctx, stream, sampler, integrand, width, height, counts, 0u, 0xFFFFFFFFu, loss, means,
                            target, grad_params, workspace, workspace_bytes, 2);
}

extern "C" qmc_status qmc_sample_offsets(qmc_context ctx, qmc_stream stream, const uint32_t* counts,
                                         uint32_t num_pixels, uint64_t* offsets, void* workspace,
                                         size_t workspace_bytes) {
    const char* who = "qmc_sample_offsets";
    if (!ctx || !counts || !offsets || !workspace) return fail(QMC_ERR_INVALID_ARGUMENT, "%s: NULL argument", who);
    if (num_pixels == 0) return fail(QMC_ERR_INVALID_ARGUMENT, "%s: num_pixels is 0", who);
    const uint32_t nblocks = (num_pixels + 1023) / 1024;
    if (workspace_bytes < size_t(nblocks) * 8)
        return fail(QMC_ERR_WORKSPACE, "%s: workspace of %zu bytes needed", who, size_t(nblocks) * 8);
    DeviceGuard guard(ctx->device);
    if (guard.status != QMC_OK) return guard.status;
    hipStream_t hs = as_stream(stream);
    uint64_t* tot = static_cast<uint64_t*>(workspace);
    clear_launch_error();
    hipLaunchKernelGGL(scan_blocks, dim3(nblocks), dim3(256), 0, hs, counts, num_pixels, offsets, tot);
    hipLaunchKernelGGL(scan_totals, dim3(1), dim3(64), 0, hs, tot, nblocks, offsets, num_pixels);
    hipLaunchKernelGGL(scan_add, dim3((num_pixels + 255) / 256), dim3(256), 0, hs, offsets, num_pixels, tot);
    return check_launch(who);
}

extern "C" qmc_status qmc_generate_pixel_samples(qmc_context ctx, qmc_stream stream, const qmc_sampler* sampler,
                                                 uint32_t d, uint32_t width, uint32_t height, const uint32_t* counts,
                                                 const uint64_t* offsets, float* out, uint64_t ld,
                                                 void* workspace, size_t workspace_bytes) {
    const char* who = "qmc_generate_pixel_samples";
    if (!ctx || !sampler || !counts || !offsets || !out) return fail(QMC_ERR_INVALID_ARGUMENT, "%s: NULL argument", who);
    if (sampler->kind == QMC_SAMPLER_POINTS) return fail(QMC_ERR_INVALID_ARGUMENT, "%s: sampler must generate", who);
    if (d == 0 || d > QMC_MAX_DIMS) return fail(QMC_ERR_OUT_OF_RANGE, "%s: d out of range", who);
    qmc_status st = validate_sampler(who, sampler, d);
    if (st == QMC_OK) st = validate_hilbert(who, sampler, width, height);
    if (st != QMC_OK) return st;
    if (uint64_t(width) * height == 0 || uint64_t(width) * height > 0xFFFFFFFFull - kTile)
        return fail(QMC_ERR_OUT_OF_RANGE, "%s: image size out of range", who);
    if (!workspace || workspace_bytes < kQueueBytes)
        return fail(QMC_ERR_WORKSPACE, "%s: %zu bytes of workspace needed", who, kQueueBytes);
    DeviceGuard guard(ctx->device);
    if (guard.status != QMC_OK) return guard.status;
    hipStream_t hs = as_stream(stream);
    const uint32_t P = width * height;
    Args a = base_args(sampler, d, width, height, counts, 0u, 0xFFFFFFFFu);
    a.offsets = offsets;
    a.out = out;
    a.out_ld = ld;
    a.queue = static_cast<uint32_t*>(workspace);
    IntegrateTune tn;
    const uint32_t grid = persistent_grid(ctx, tn, a.num_tasks, &a);
    const bool nus = (sampler->flags & QMC_PIXEL_NUS) != 0, shift = (sampler->flags & QMC_PIXEL_SHIFT) != 0;
    const bool back = (sampler->flags & QMC_LATTICE_BACKWARD) != 0;
    clear_launch_error();
    if (a.dynamic) hipLaunchKernelGGL(reset_queue, dim3(1), dim3(kWave), 0, hs, a.queue);
    if (d <= 8)
        dispatch_sampler<SamplesFam<8>>(sampler->kind, nus, shift, back, grid, hs, a);
    else
        dispatch_sampler<SamplesFam<QMC_MAX_DIMS>>(sampler->kind, nus, shift, back, grid, hs, a);
    return check_launch(who);
}

extern "C" qmc_status qmc_integrate_pixels_l2_step_noalloc(qmc_context ctx, qmc_stream stream,
                                                           const qmc_sampler* sampler, const qmc_integrand* integrand,
                                                           uint32_t width, uint32_t height, const uint32_t* counts,
                                                           const float* target, float* means, float* loss,
                                                           float* grad_params) {
    const char* who = "qmc_integrate_pixels_l2_step_noalloc";
    if (!ctx || !sampler || !integrand || !loss)
        return fail(QMC_ERR_INVALID_ARGUMENT, "%s: NULL context, sampler, integrand or loss", who);
    if (!ctx->static_scratch) return fail(QMC_ERR_DEVICE, "%s: the context has no static scratch", who);
    const size_t need = make_plan(integrand, width * height, 2).total;
    if (need > QMC_STATIC_SCRATCH_BYTES)
        return fail(QMC_ERR_WORKSPACE, "%s: the problem needs %zu bytes of scratch, the static scratch holds %u "
                    "(at most 6550 parameters)", who, need, QMC_STATIC_SCRATCH_BYTES);
    return integrate_common(who, ctx, stream, sampler, integrand, width, height, counts, 0u, 0xFFFFFFFFu, loss, means,
                            target, grad_params, ctx->static_scratch, QMC_STATIC_SCRATCH_BYTES, 2);
}
