// Materialised point generation: digital sequences (Sec. 2.3, Eq. ts) and rank-1 lattice
// sequences (Sec. 2.4, Eq. R1LS), randomised in integers and converted by
// map_u32_to_unifloat (Sec. 2.1, Alg. 1).
//
// Output is dimension-major, out[j*ld + (i - first)].  The fast kernels give each lane four
// consecutive indices, so a wavefront writes 256 consecutive u32 (1 KiB) per dimension with
// 16-byte stores, and each wavefront owns a run of such 256-index chunks.  For one
// dimension the run is generated with a single register of state:
//   * the first point of the run is the plain matrix product (one select-XOR per index bit);
//   * the four indices 4q..4q+3 of a lane differ only in bits 0 and 1, so their points are
//     x, x^C[0], x^C[1], x^C[0]^C[1];
//   * moving a lane from index i to i+256 flips index bits 8..8+t, t = ctz((i>>8)+1), so
//     x(i+256) = x(i) ^ Q[t] with Q[t] = C[8]^...^C[8+t], a table built once per block.
// With scrambling the columns are staged bit-reversed, which yields the mirrored value the
// nested scramble starts from at no cost.  Every kernel here switches its wavefronts to
// round-toward-zero FP32 rounding on entry, so the float conversion is the hardware
// u32 -> f32 conversion (which then truncates) followed by an exact scaling by 2^-32.
#include "common.hpp"
#include "device_core.hpp"

namespace qmc {
namespace {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr uint32_t kBlock = 256;
constexpr uint32_t kWavesPerBlock = kBlock / 64;
constexpr uint32_t kChunk = 256;  // indices per wavefront step
constexpr uint32_t kQ = 24;       // stride-table entries per dimension (index bits 8..31)

template <bool NT, typename V>
__device__ __forceinline__ void store_vec(V* p, V v) {
    if constexpr (NT)
        __builtin_nontemporal_store(v, p);
    else
        *p = v;
}

template <bool NT, typename T>
__device__ __forceinline__ void store_one(T* p, T v) {
    if constexpr (NT)
        __builtin_nontemporal_store(v, p);
    else
        *p = v;
}

// Final integer stage shared by both sequence kinds: shift, then store u32 and/or float.
template <bool SHIFT, bool SXOR, bool WU, bool WF, bool NT>
__device__ __forceinline__ void emit4(uint32_t* ou, float* of, uint64_t off, uint32_t valid, uint32_t r0,
                                      uint32_t r1, uint32_t r2, uint32_t r3, uint32_t sh) {
    if constexpr (SHIFT) {
        r0 = dev::apply_shift<SXOR>(r0, sh);
        r1 = dev::apply_shift<SXOR>(r1, sh);
        r2 = dev::apply_shift<SXOR>(r2, sh);
        r3 = dev::apply_shift<SXOR>(r3, sh);
    }
    if (valid >= 4) {
        if constexpr (WU) store_vec<NT>(reinterpret_cast<u32x4*>(ou + off), u32x4{r0, r1, r2, r3});
        if constexpr (WF)
            store_vec<NT>(reinterpret_cast<f32x4*>(of + off),
                          f32x4{dev::u32_to_unifloat_rtz(r0), dev::u32_to_unifloat_rtz(r1), dev::u32_to_unifloat_rtz(r2),
                                dev::u32_to_unifloat_rtz(r3)});
    } else {
        const uint32_t r[4] = {r0, r1, r2, r3};
        for (uint32_t q = 0; q < valid; ++q) {
            if constexpr (WU) store_one<NT>(ou + off + q, r[q]);
            if constexpr (WF) store_one<NT>(of + off + q, dev::u32_to_unifloat_rtz(r[q]));
        }
    }
}

struct SobolLds {
    uint32_t cols[QMC_MAX_DIMS][32];
    uint32_t q[QMC_MAX_DIMS][kQ];
    uint32_t seed[QMC_MAX_DIMS];
    uint32_t sm[QMC_MAX_DIMS];
    uint32_t shift[QMC_MAX_DIMS];
};

// Q[j][t] = XOR of columns q0..q0+t of dimension j: moving an index by 2^q0 flips its bits
// q0..q0+t with t = ctz((i >> q0) + 1), so the point moves by Q[j][t].
template <bool NUS, bool SHIFT>
__device__ __forceinline__ void stage_sobol(SobolLds& L, const uint32_t* __restrict__ mats, uint32_t s,
                                            const uint32_t* __restrict__ seeds, const uint32_t* __restrict__ shifts,
                                            bool build_q, uint32_t q0 = 8) {
    const uint32_t tid = threadIdx.x;
    for (uint32_t t = tid; t < s * 32; t += blockDim.x) {
        const uint32_t c = mats[t];
        L.cols[t >> 5][t & 31] = NUS ? dev::brev(c) : c;
    }
    for (uint32_t t = tid; t < s; t += blockDim.x) {
        if constexpr (NUS) {
            L.seed[t] = seeds[t];
            L.sm[t] = dev::seed_multiplier(seeds[t]);
        }
        if constexpr (SHIFT) L.shift[t] = shifts[t];
    }
    __syncthreads();
    if (build_q) {
        for (uint32_t t = tid; t < s * kQ; t += blockDim.x) {
            const uint32_t j = t / kQ, k = t % kQ;
            uint32_t acc = 0;
            for (uint32_t b = 0; b <= k && q0 + b < 32; ++b) acc ^= L.cols[j][q0 + b];
            L.q[j][k] = acc;
        }
        __syncthreads();
    }
}

__device__ __forceinline__ uint32_t matrix_product(const uint32_t* cols, uint32_t i) {
    uint32_t x = 0;
#pragma unroll
    for (int k = 0; k < 32; ++k) x ^= ((i >> k) & 1u) ? cols[k] : 0u;
    return x;
}

// Chunk order: wavefront w handles chunks c0 + k * step for k < steps, where
//   contiguous runs: c0 = w * steps, step = 1;
//   interleaved:     c0 = w, step = W (all wavefronts, a power of two), so at every step the
//                    whole grid writes one contiguous window of W chunks per output array.
// step * 256 = 2^q0 indices, and the Q table is built from column q0.
template <bool NUS, bool SHIFT, bool SXOR, bool WU, bool WF, bool NT>
__global__ __launch_bounds__(kBlock) void sobol_fast(const uint32_t* __restrict__ mats, uint32_t s, uint32_t first,
                                                     uint32_t n, const uint32_t* __restrict__ seeds,
                                                     const uint32_t* __restrict__ shifts, uint32_t* __restrict__ ou,
                                                     float* __restrict__ of, uint64_t ld, uint32_t steps,
                                                     uint32_t nchunks, uint32_t interleaved, uint32_t q0) {
    dev::set_fp32_round_toward_zero();
    __shared__ SobolLds L;
    stage_sobol<NUS, SHIFT>(L, mats, s, seeds, shifts, true, q0);
    const uint32_t wave = blockIdx.x * kWavesPerBlock + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t step = interleaved ? gridDim.x * kWavesPerBlock : 1u;
    const uint32_t c0 = interleaved ? wave : wave * steps;
    if (c0 >= nchunks) return;
    const uint32_t kmax = interleaved ? (nchunks - c0 + step - 1) / step : min(steps, nchunks - c0);
    const uint32_t full = n / kChunk;  // chunks with all 256 indices in range
    const uint32_t stride = step * kChunk;
    for (uint32_t j = 0; j < s; ++j) {
        uint32_t c = c0;
        uint32_t o = c0 * kChunk + 4u * lane;
        uint32_t i = first + o;
        uint32_t x = matrix_product(L.cols[j], i);
        const uint32_t col0 = L.cols[j][0], col1 = L.cols[j][1];
        const uint32_t seed = NUS ? L.seed[j] : 0u, sm = NUS ? L.sm[j] : 0u;
        const uint32_t sh = SHIFT ? L.shift[j] : 0u;
        const uint64_t base = uint64_t(j) * ld;
        for (uint32_t k = 0; k < kmax; ++k) {
            uint32_t v0 = x, v1 = x ^ col0, v2 = x ^ col1, v3 = x ^ col0 ^ col1;
            if constexpr (NUS) {
                v0 = dev::nus_from_mirrored(v0, seed, sm);
                v1 = dev::nus_from_mirrored(v1, seed, sm);
                v2 = dev::nus_from_mirrored(v2, seed, sm);
                v3 = dev::nus_from_mirrored(v3, seed, sm);
            }
            if (c < full)
                emit4<SHIFT, SXOR, WU, WF, NT>(ou, of, base + o, 4u, v0, v1, v2, v3, sh);
            else if (o < n)
                emit4<SHIFT, SXOR, WU, WF, NT>(ou, of, base + o, min(n - o, 4u), v0, v1, v2, v3, sh);
            if (k + 1 < kmax) {
                const uint32_t t = min(static_cast<uint32_t>(__builtin_ctz((i >> q0) + 1u)), kQ - 1);
                x ^= L.q[j][t];
                i += stride;
                o += stride;
                c += step;
            }
        }
    }
}

// Any alignment: one index per thread, each point from the plain matrix product.
template <bool NUS, bool SHIFT, bool SXOR, bool WU, bool WF>
__global__ __launch_bounds__(kBlock) void sobol_general(const uint32_t* __restrict__ mats, uint32_t s, uint32_t first,
                                                        uint32_t n, const uint32_t* __restrict__ seeds,
                                                        const uint32_t* __restrict__ shifts, uint32_t* __restrict__ ou,
                                                        float* __restrict__ of, uint64_t ld) {
    dev::set_fp32_round_toward_zero();
    __shared__ SobolLds L;
    stage_sobol<NUS, SHIFT>(L, mats, s, seeds, shifts, false);
    for (uint32_t o = blockIdx.x * kBlock + threadIdx.x; o < n; o += gridDim.x * kBlock) {
        const uint32_t i = first + o;
        for (uint32_t j = 0; j < s; ++j) {
            uint32_t v = matrix_product(L.cols[j], i);
            if constexpr (NUS) v = dev::nus_from_mirrored(v, L.seed[j], L.sm[j]);
            if constexpr (SHIFT) v = dev::apply_shift<SXOR>(v, L.shift[j]);
            if constexpr (WU) ou[uint64_t(j) * ld + o] = v;
            if constexpr (WF) of[uint64_t(j) * ld + o] = dev::u32_to_unifloat_rtz(v);
        }
    }
}

struct LatticeLds {
    uint32_t g[QMC_MAX_DIMS];
    uint32_t shift[QMC_MAX_DIMS];
};

template <bool SHIFT>
__device__ __forceinline__ void stage_lattice(LatticeLds& L, const uint32_t* __restrict__ gen, uint32_t s,
                                              const uint32_t* __restrict__ shifts) {
    for (uint32_t t = threadIdx.x; t < s; t += blockDim.x) {
        L.g[t] = gen[t];
        if constexpr (SHIFT) L.shift[t] = shifts[t];
    }
    __syncthreads();
}

// brev(i + r) = brev(i) | brev(r) for i % 4 == 0 and r < 4, so the four points of a lane are
// x0 + brev(r) g (forward) or x0 - brev(r) g with x0 = ~brev(i) g (backward), brev(1) = 2^31,
// brev(2) = 2^30.
template <bool BACK, bool SHIFT, bool SXOR, bool WU, bool WF, bool NT>
__global__ __launch_bounds__(kBlock) void lattice_fast(const uint32_t* __restrict__ gen, uint32_t s, uint32_t first,
                                                       uint32_t n, const uint32_t* __restrict__ shifts,
                                                       uint32_t* __restrict__ ou, float* __restrict__ of, uint64_t ld,
                                                       uint32_t cpw, uint32_t nchunks, uint32_t interleaved) {
    dev::set_fp32_round_toward_zero();
    __shared__ LatticeLds L;
    stage_lattice<SHIFT>(L, gen, s, shifts);
    const uint32_t wave = blockIdx.x * kWavesPerBlock + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t step = interleaved ? gridDim.x * kWavesPerBlock : 1u;
    const uint32_t c0 = interleaved ? wave : wave * cpw;
    if (c0 >= nchunks) return;
    const uint32_t kmax = interleaved ? (nchunks - c0 + step - 1) / step : min(cpw, nchunks - c0);
    const uint32_t full = n / kChunk;
    for (uint32_t j = 0; j < s; ++j) {
        const uint32_t g = L.g[j];
        const uint32_t h1 = g << 31, h2 = g << 30, h3 = h1 + h2;
        const uint32_t sh = SHIFT ? L.shift[j] : 0u;
        const uint64_t base = uint64_t(j) * ld;
        for (uint32_t k = 0; k < kmax; ++k) {
            const uint32_t c = c0 + k * step;
            const uint32_t o = c * kChunk + 4u * lane;
            if (c >= full && o >= n) break;
            const uint32_t b = dev::brev(first + o);
            uint32_t v0, v1, v2, v3;
            if constexpr (BACK) {
                v0 = (~b) * g;
                v1 = v0 - h1;
                v2 = v0 - h2;
                v3 = v0 - h3;
            } else {
                v0 = b * g;
                v1 = v0 + h1;
                v2 = v0 + h2;
                v3 = v0 + h3;
            }
            if (c < full)
                emit4<SHIFT, SXOR, WU, WF, NT>(ou, of, base + o, 4u, v0, v1, v2, v3, sh);
            else
                emit4<SHIFT, SXOR, WU, WF, NT>(ou, of, base + o, min(n - o, 4u), v0, v1, v2, v3, sh);
        }
    }
}

template <bool BACK, bool SHIFT, bool SXOR, bool WU, bool WF>
__global__ __launch_bounds__(kBlock) void lattice_general(const uint32_t* __restrict__ gen, uint32_t s, uint32_t first,
                                                          uint32_t n, const uint32_t* __restrict__ shifts,
                                                          uint32_t* __restrict__ ou, float* __restrict__ of,
                                                          uint64_t ld) {
    dev::set_fp32_round_toward_zero();
    __shared__ LatticeLds L;
    stage_lattice<SHIFT>(L, gen, s, shifts);
    for (uint32_t o = blockIdx.x * kBlock + threadIdx.x; o < n; o += gridDim.x * kBlock) {
        const uint32_t i = first + o;
        const uint32_t b = dev::brev(BACK ? ~i : i);
        for (uint32_t j = 0; j < s; ++j) {
            uint32_t v = b * L.g[j];
            if constexpr (SHIFT) v = dev::apply_shift<SXOR>(v, L.shift[j]);
            if constexpr (WU) ou[uint64_t(j) * ld + o] = v;
            if constexpr (WF) of[uint64_t(j) * ld + o] = dev::u32_to_unifloat_rtz(v);
        }
    }
}

__global__ __launch_bounds__(kBlock) void unifloat_vec(const u32x4* __restrict__ in, f32x4* __restrict__ out,
                                                       uint64_t nvec) {
    dev::set_fp32_round_toward_zero();
    for (uint64_t k = uint64_t(blockIdx.x) * kBlock + threadIdx.x; k < nvec; k += uint64_t(gridDim.x) * kBlock) {
        const u32x4 u = in[k];
        out[k] = f32x4{dev::u32_to_unifloat_rtz(u.x), dev::u32_to_unifloat_rtz(u.y), dev::u32_to_unifloat_rtz(u.z),
                       dev::u32_to_unifloat_rtz(u.w)};
    }
}

__global__ __launch_bounds__(kBlock) void unifloat_scalar(const uint32_t* __restrict__ in, float* __restrict__ out,
                                                          uint64_t begin, uint64_t n) {
    dev::set_fp32_round_toward_zero();
    for (uint64_t k = begin + uint64_t(blockIdx.x) * kBlock + threadIdx.x; k < n; k += uint64_t(gridDim.x) * kBlock)
        out[k] = dev::u32_to_unifloat_rtz(in[k]);
}

template <typename F>
void with_bool(bool b, F&& f) {
    if (b)
        f(std::true_type{});
    else
        f(std::false_type{});
}

// Which outputs are written: both, u32 only or float only.
template <typename F>
void with_outputs(bool wu, bool wf, F&& f) {
    if (wu && wf)
        f(std::true_type{}, std::true_type{});
    else if (wu)
        f(std::true_type{}, std::false_type{});
    else
        f(std::false_type{}, std::true_type{});
}

bool ranges_overlap(const void* a, uint64_t abytes, const void* b, uint64_t bbytes) {
    if (!a || !b || !abytes || !bbytes) return false;
    const uintptr_t a0 = reinterpret_cast<uintptr_t>(a), b0 = reinterpret_cast<uintptr_t>(b);
    return a0 < b0 + bbytes && b0 < a0 + abytes;
}

// Shared validation of the generation calls.
qmc_status validate_generation(const char* who, qmc_context ctx, const void* table, uint64_t table_bytes_per_dim,
                               uint32_t s, uint64_t first, uint64_t n, uint32_t flags, uint32_t allowed_flags,
                               const void* aux0, const void* aux1, const uint32_t* ou, const float* of, uint64_t ld) {
    if (!ctx) return fail(QMC_ERR_INVALID_ARGUMENT, "%s: context is NULL", who);
    if (s == 0 || s > QMC_MAX_DIMS) return fail(QMC_ERR_OUT_OF_RANGE, "%s: s = %u outside [1, %d]", who, s, QMC_MAX_DIMS);
    if (first > (uint64_t(1) << 32) || n > (uint64_t(1) << 32) - first)
        return fail(QMC_ERR_OUT_OF_RANGE, "%s: first + n exceeds 2^32 (first=%llu n=%llu)", who,
                    (unsigned long long)first, (unsigned long long)n);
    if (flags & ~allowed_flags) return fail(QMC_ERR_INVALID_ARGUMENT, "%s: unknown flags 0x%x", who, flags);
    if (n == 0) return QMC_OK;
    if (!table) return fail(QMC_ERR_INVALID_ARGUMENT, "%s: table pointer is NULL", who);
    if (!ou && !of) return fail(QMC_ERR_INVALID_ARGUMENT, "%s: both outputs are NULL", who);
    if (ld < n) return fail(QMC_ERR_INVALID_ARGUMENT, "%s: ld (%llu) < n (%llu)", who, (unsigned long long)ld,
                            (unsigned long long)n);
    if (ld > (uint64_t(1) << 56) / s) return fail(QMC_ERR_OUT_OF_RANGE, "%s: ld too large", who);
    const uint64_t out_bytes = ((uint64_t(s) - 1) * ld + n) * 4;
    if (ranges_overlap(ou, out_bytes, of, out_bytes))
        return fail(QMC_ERR_INVALID_ARGUMENT, "%s: outputs overlap", who);
    const void* ins[3] = {table, aux0, aux1};
    const uint64_t in_bytes[3] = {uint64_t(s) * table_bytes_per_dim, uint64_t(s) * 4, uint64_t(s) * 4};
    for (int k = 0; k < 3; ++k)
        if (ranges_overlap(ins[k], in_bytes[k], ou, out_bytes) || ranges_overlap(ins[k], in_bytes[k], of, out_bytes))
            return fail(QMC_ERR_INVALID_ARGUMENT, "%s: an output overlaps an input", who);
    return QMC_OK;
}

// Grid of the fast kernels.  Contiguous runs: one wavefront per `cpw` chunks.  Interleaved:
// a power-of-two number of wavefronts (at most tune.waves, at most one per chunk), so that the
// index stride between a wavefront's chunks is a power of two.
uint32_t fast_grid(uint64_t n, const GenTune& tn, uint32_t* nchunks, uint32_t* q0) {
    *nchunks = static_cast<uint32_t>((n + kChunk - 1) / kChunk);
    if (!tn.interleaved) {
        *q0 = 8;
        const uint32_t waves = (*nchunks + tn.chunks_per_wave - 1) / tn.chunks_per_wave;
        return (waves + kWavesPerBlock - 1) / kWavesPerBlock;
    }
    uint32_t waves = kWavesPerBlock;
    while (waves * 2 <= tn.waves && waves * 2 <= *nchunks) waves *= 2;
    uint32_t lg = 0;
    while ((1u << lg) < waves) ++lg;
    *q0 = 8 + lg;
    return waves / kWavesPerBlock;
}

uint32_t general_grid(const qmc_context ctx, uint64_t n) {
    const uint64_t want = (n + kBlock - 1) / kBlock;
    const uint64_t cap = uint64_t(ctx->num_cus) * 8;
    return static_cast<uint32_t>(want < cap ? want : cap);
}

}  // namespace
}  // namespace qmc

using namespace qmc;

extern "C" qmc_status qmc_generate_sobol(qmc_context ctx, qmc_stream stream, const uint32_t* matrices, uint32_t s,
                                         uint64_t first, uint64_t n, const uint32_t* nus_seeds,
                                         const uint32_t* shifts, uint32_t flags, uint32_t* out_u32, float* out_f32,
                                         uint64_t ld) {
    const char* who = "qmc_generate_sobol";
    qmc_status st = validate_generation(who, ctx, matrices, 128, s, first, n, flags, QMC_SHIFT_XOR, nus_seeds, shifts,
                                        out_u32, out_f32, ld);
    if (st != QMC_OK || n == 0) return st;
    if (n > (uint64_t(1) << 31)) {  // kernels count indices in 32 bits: split [0, 2^32)
        const uint64_t h = uint64_t(1) << 31;
        st = qmc_generate_sobol(ctx, stream, matrices, s, first, h, nus_seeds, shifts, flags, out_u32, out_f32, ld);
        if (st != QMC_OK) return st;
        return qmc_generate_sobol(ctx, stream, matrices, s, first + h, n - h, nus_seeds, shifts, flags,
                                  out_u32 ? out_u32 + h : nullptr, out_f32 ? out_f32 + h : nullptr, ld);
    }
    DeviceGuard guard(ctx->device);
    if (guard.status != QMC_OK) return guard.status;
    hipStream_t hs = as_stream(stream);
    const bool nus = nus_seeds != nullptr, shift = shifts != nullptr, sxor = (flags & QMC_SHIFT_XOR) != 0;
    const bool fast = (first % 4 == 0) && (ld % 4 == 0) && aligned16(out_u32) && aligned16(out_f32);
    const uint32_t first32 = static_cast<uint32_t>(first);  // first < 2^32 whenever n > 0
    const uint32_t nn = static_cast<uint32_t>(n);
    clear_launch_error();
    with_bool(nus, [&](auto NUS) {
        with_bool(shift, [&](auto SH) {
            with_bool(sxor && shift, [&](auto SX) {
                with_outputs(out_u32 != nullptr, out_f32 != nullptr, [&](auto WU, auto WF) {
                    if (fast) {
                        with_bool(ctx->sobol_tune.nontemporal != 0, [&](auto NT) {
                            uint32_t nchunks, q0;
                            const GenTune& tn = ctx->sobol_tune;
                            const uint32_t grid = fast_grid(nn, tn, &nchunks, &q0);
                            hipLaunchKernelGGL((sobol_fast<NUS.value, SH.value, SX.value, WU.value, WF.value, NT.value>),
                                               dim3(grid), dim3(kBlock), 0, hs, matrices, s, first32, nn, nus_seeds,
                                               shifts, out_u32, out_f32, ld, tn.chunks_per_wave, nchunks,
                                               tn.interleaved, q0);
                        });
                    } else {
                        hipLaunchKernelGGL((sobol_general<NUS.value, SH.value, SX.value, WU.value, WF.value>),
                                           dim3(general_grid(ctx, nn)), dim3(kBlock), 0, hs, matrices, s, first32, nn,
                                           nus_seeds, shifts, out_u32, out_f32, ld);
                    }
                });
            });
        });
    });
    return check_launch(who);
}

extern "C" qmc_status qmc_generate_lattice(qmc_context ctx, qmc_stream stream, const uint32_t* generator, uint32_t s,
                                           uint64_t first, uint64_t n, const uint32_t* shifts, uint32_t flags,
                                           uint32_t* out_u32, float* out_f32, uint64_t ld) {
    const char* who = "qmc_generate_lattice";
    qmc_status st = validate_generation(who, ctx, generator, 4, s, first, n, flags,
                                        QMC_SHIFT_XOR | QMC_LATTICE_BACKWARD, shifts, nullptr, out_u32, out_f32, ld);
    if (st != QMC_OK || n == 0) return st;
    if (n > (uint64_t(1) << 31)) {  // kernels count indices in 32 bits: split [0, 2^32)
        const uint64_t h = uint64_t(1) << 31;
        st = qmc_generate_lattice(ctx, stream, generator, s, first, h, shifts, flags, out_u32, out_f32, ld);
        if (st != QMC_OK) return st;
        return qmc_generate_lattice(ctx, stream, generator, s, first + h, n - h, shifts, flags,
                                    out_u32 ? out_u32 + h : nullptr, out_f32 ? out_f32 + h : nullptr, ld);
    }
    DeviceGuard guard(ctx->device);
    if (guard.status != QMC_OK) return guard.status;
    hipStream_t hs = as_stream(stream);
    const bool back = (flags & QMC_LATTICE_BACKWARD) != 0, shift = shifts != nullptr;
    const bool sxor = (flags & QMC_SHIFT_XOR) != 0;
    const bool fast = (first % 4 == 0) && (ld % 4 == 0) && aligned16(out_u32) && aligned16(out_f32);
    const uint32_t first32 = static_cast<uint32_t>(first);
    const uint32_t nn = static_cast<uint32_t>(n);
    clear_launch_error();
    with_bool(back, [&](auto BK) {
        with_bool(shift, [&](auto SH) {
            with_bool(sxor && shift, [&](auto SX) {
                with_outputs(out_u32 != nullptr, out_f32 != nullptr, [&](auto WU, auto WF) {
                    if (fast) {
                        with_bool(ctx->lattice_tune.nontemporal != 0, [&](auto NT) {
                            uint32_t nchunks, q0;
                            const GenTune& tn = ctx->lattice_tune;
                            const uint32_t grid = fast_grid(nn, tn, &nchunks, &q0);
                            hipLaunchKernelGGL(
                                (lattice_fast<BK.value, SH.value, SX.value, WU.value, WF.value, NT.value>),
                                dim3(grid), dim3(kBlock), 0, hs, generator, s, first32, nn, shifts, out_u32, out_f32,
                                ld, tn.chunks_per_wave, nchunks, tn.interleaved);
                        });
                    } else {
                        hipLaunchKernelGGL((lattice_general<BK.value, SH.value, SX.value, WU.value, WF.value>),
                                           dim3(general_grid(ctx, nn)), dim3(kBlock), 0, hs, generator, s, first32,
                                           nn, shifts, out_u32, out_f32, ld);
                    }
                });
            });
        });
    });
    return check_launch(who);
}

extern "C" qmc_status qmc_map_u32_to_unifloat(qmc_context ctx, qmc_stream stream, const uint32_t* in, float* out,
                                              uint64_t n) {
    const char* who = "qmc_map_u32_to_unifloat";
    if (!ctx) return fail(QMC_ERR_INVALID_ARGUMENT, "%s: context is NULL", who);
    if (n == 0) return QMC_OK;
    if (!in || !out) return fail(QMC_ERR_INVALID_ARGUMENT, "%s: NULL pointer", who);
    if (reinterpret_cast<const void*>(in) != reinterpret_cast<const void*>(out) && ranges_overlap(in, n * 4, out, n * 4))
        return fail(QMC_ERR_INVALID_ARGUMENT, "%s: in and out overlap partially", who);
    DeviceGuard guard(ctx->device);
    if (guard.status != QMC_OK) return guard.status;
    hipStream_t hs = as_stream(stream);
    clear_launch_error();
    uint64_t done = 0;
    const uint64_t cap = uint64_t(ctx->num_cus) * 16;
    if (aligned16(in) && aligned16(out)) {
        const uint64_t nvec = n / 4;
        if (nvec) {
            const uint64_t want = (nvec + kBlock - 1) / kBlock;
            hipLaunchKernelGGL(unifloat_vec, dim3(static_cast<uint32_t>(want < cap ? want : cap)), dim3(kBlock), 0, hs,
                               reinterpret_cast<const u32x4*>(in), reinterpret_cast<f32x4*>(out), nvec);
        }
        done = nvec * 4;
    }
    if (done < n) {
        const uint64_t want = (n - done + kBlock - 1) / kBlock;
        hipLaunchKernelGGL(unifloat_scalar, dim3(static_cast<uint32_t>(want < cap ? want : cap)), dim3(kBlock), 0, hs,
                           in, out, done, n);
    }
    return check_launch(who);
}
