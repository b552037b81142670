// Materialised point generation: digital sequences (Sec. 2.3, Eq. ts) and rank-1 lattice
// sequences (Sec. 2.4, Eq. R1LS), randomised in integers and converted by
// map_u32_to_unifloat (Sec. 2.1, Alg. 1); the same with 64-bit indices and partitioned
// enumeration (Sec. 2.5.1); point-major output; the Halton sequence (Sec. 2.2).
//
// Output is dimension-major, out[j*ld + (i - first)], unless the point-major layout is asked
// for (its kernels are described with them).  The fast kernels launch one wavefront
// per (dimension, run of `cpw` chunks of 256 indices), in dimension-major order, so that the
// wavefronts in flight at any moment write one narrow, advancing window of each output array:
// the access order of a plain fill, which is what the HBM write path sustains best.  Each lane
// takes four consecutive indices and writes them with one 16-byte store per output array.
//
// For a digital sequence the point of index i is the XOR of the columns selected by the bits
// of i.  With i = 256 h + t (t the lane's offset within the chunk, bits 0..7 after the carry
// is split off):
//   * the part from bits 8..31 (the chunk, wave-uniform) is formed by lanes 8..31 each
//     contributing one column, then an XOR reduction across the half-wavefront; the other
//     half-wavefront forms the part for h + 1, needed by lanes whose offset carries into bit 8
//     when `first` is not a multiple of 256;
//   * the part from bits 2..7 is fixed per lane and formed once;
//   * the four indices of a lane differ in bits 0 and 1: x, x^C[0], x^C[1], x^C[0]^C[1].
// With scrambling the columns are bit-reversed first, which yields the mirrored value the
// nested scramble starts from at no cost.  Every kernel here switches its wavefronts to
// round-toward-zero FP32 rounding on entry, so the float conversion is the hardware
// u32 -> f32 conversion (which then truncates) followed by an exact scaling by 2^-32.
#include "common.hpp"
#include "device_core.hpp"

namespace qmc {
namespace {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr uint32_t kBlock = 256;  // block size of the general (any alignment) kernels
constexpr uint32_t kWave = 64;    // the fast kernels run one wavefront per block
constexpr uint32_t kChunk = 256;  // indices per wavefront step

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
    uint32_t seed[QMC_MAX_DIMS];
    uint32_t sm[QMC_MAX_DIMS];
    uint32_t shift[QMC_MAX_DIMS];
};

template <bool NUS, bool SHIFT>
__device__ __forceinline__ void stage_sobol(SobolLds& L, const uint32_t* __restrict__ mats, uint32_t s,
                                            const uint32_t* __restrict__ seeds, const uint32_t* __restrict__ shifts) {
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
}

__device__ __forceinline__ uint32_t matrix_product(const uint32_t* cols, uint32_t i) {
    uint32_t x = 0;
#pragma unroll
    for (int k = 0; k < 32; ++k) x ^= ((i >> k) & 1u) ? cols[k] : 0u;
    return x;
}

// XOR of v over the 32 lanes of each half-wavefront, returned to lanes 31 and 63 (other lanes
// receive partial sums).  DPP: XOR within quads, across the quads of each row of 16 lanes
// (rotations by 4 and 8), then row 0 (2) into row 1 (3) with a broadcast of lane 15.
__device__ __forceinline__ uint32_t half_wave_xor(uint32_t v) {
    const int x = static_cast<int>(v);
    int r = x ^ __builtin_amdgcn_update_dpp(0, x, 0xB1, 0xF, 0xF, false);   // quad_perm [1,0,3,2]
    r ^= __builtin_amdgcn_update_dpp(0, r, 0x4E, 0xF, 0xF, false);          // quad_perm [2,3,0,1]
    r ^= __builtin_amdgcn_update_dpp(0, r, 0x124, 0xF, 0xF, false);         // row_ror 4
    r ^= __builtin_amdgcn_update_dpp(0, r, 0x128, 0xF, 0xF, false);         // row_ror 8
    r ^= __builtin_amdgcn_update_dpp(0, r, 0x142, 0xA, 0xF, false);         // row_bcast 15 into rows 1, 3
    return static_cast<uint32_t>(r);
}

// Block (x, j): dimension j, chunks [x * cpw, min((x + 1) * cpw, nchunks)).  Needs first % 4 == 0,
// ld % 4 == 0 and 16-byte aligned outputs; n <= 2^31 and first + n <= 2^32.
template <bool NUS, bool SHIFT, bool SXOR, bool WU, bool WF, bool NT>
__global__ __launch_bounds__(kWave) void sobol_fast(const uint32_t* __restrict__ mats, uint32_t first, uint32_t n,
                                                    const uint32_t* __restrict__ seeds,
                                                    const uint32_t* __restrict__ shifts, uint32_t* __restrict__ ou,
                                                    float* __restrict__ of, uint64_t ld, uint32_t cpw,
                                                    uint32_t nchunks) {
    dev::set_fp32_round_toward_zero();
    const uint32_t j = blockIdx.y;
    const uint32_t lane = threadIdx.x;
    const uint32_t cb = blockIdx.x * cpw;
    const uint32_t ce = min(cb + cpw, nchunks);
    uint32_t col = mats[j * 32 + (lane & 31)];  // lane k (and k + 32) holds column k
    if constexpr (NUS) col = dev::brev(col);
    const uint32_t seed = NUS ? seeds[j] : 0u;
    const uint32_t sm = dev::seed_multiplier(seed);
    const uint32_t sh = SHIFT ? shifts[j] : 0u;
    // i = first + 256 c + 4 lane + r = 256 (first/256 + c) + t + r with t = first%256 + 4 lane < 512.
    const uint32_t t = (first & 255u) + 4u * lane;
    const uint32_t carry = 0u - (t >> 8);  // all ones where the offset carries into bit 8
    uint32_t xlo = 0;
#pragma unroll
    for (int k = 2; k < 8; ++k) xlo ^= (0u - ((t >> k) & 1u)) & __builtin_amdgcn_readlane(col, k);
    const uint32_t col0 = __builtin_amdgcn_readlane(col, 0), col1 = __builtin_amdgcn_readlane(col, 1);
    const uint32_t k = lane & 31u;
    const uint64_t base = uint64_t(j) * ld;
    for (uint32_t c = cb; c < ce; ++c) {
        // Lanes 8..31 select column k for bit k of 256 h, lanes 40..63 the same for 256 (h + 1).
        const uint32_t h = (first >> 8) + c + (lane >> 5);
        const uint32_t part = half_wave_xor((k >= 8u && ((h >> (k - 8u)) & 1u)) ? col : 0u);
        const uint32_t p0 = __builtin_amdgcn_readlane(part, 31), p1 = __builtin_amdgcn_readlane(part, 63);
        const uint32_t x = (p0 ^ ((p0 ^ p1) & carry)) ^ xlo;
        uint32_t v0 = x, v1 = x ^ col0, v2 = x ^ col1, v3 = x ^ col0 ^ col1;
        if constexpr (NUS) {
            v0 = dev::nus_from_mirrored(v0, seed, sm);
            v1 = dev::nus_from_mirrored(v1, seed, sm);
            v2 = dev::nus_from_mirrored(v2, seed, sm);
            v3 = dev::nus_from_mirrored(v3, seed, sm);
        }
        const uint32_t o = c * kChunk + 4u * lane;
        if (o + 4u <= n)
            emit4<SHIFT, SXOR, WU, WF, NT>(ou, of, base + o, 4u, v0, v1, v2, v3, sh);
        else if (o < n)
            emit4<SHIFT, SXOR, WU, WF, NT>(ou, of, base + o, n - o, v0, v1, v2, v3, sh);
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
    stage_sobol<NUS, SHIFT>(L, mats, s, seeds, shifts);
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
// brev(2) = 2^30.  Block (x, j): dimension j, chunks [x * cpw, min((x + 1) * cpw, nchunks)).
template <bool BACK, bool SHIFT, bool SXOR, bool WU, bool WF, bool NT>
__global__ __launch_bounds__(kWave) void lattice_fast(const uint32_t* __restrict__ gen, uint32_t first, uint32_t n,
                                                      const uint32_t* __restrict__ shifts, uint32_t* __restrict__ ou,
                                                      float* __restrict__ of, uint64_t ld, uint32_t cpw,
                                                      uint32_t nchunks) {
    dev::set_fp32_round_toward_zero();
    const uint32_t j = blockIdx.y;
    const uint32_t lane = threadIdx.x;
    const uint32_t cb = blockIdx.x * cpw;
    const uint32_t ce = min(cb + cpw, nchunks);
    const uint32_t g = gen[j];
    const uint32_t h1 = g << 31, h2 = g << 30, h3 = h1 + h2;
    const uint32_t sh = SHIFT ? shifts[j] : 0u;
    const uint64_t base = uint64_t(j) * ld;
    for (uint32_t c = cb; c < ce; ++c) {
        const uint32_t o = c * kChunk + 4u * lane;
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
        if (o + 4u <= n)
            emit4<SHIFT, SXOR, WU, WF, NT>(ou, of, base + o, 4u, v0, v1, v2, v3, sh);
        else if (o < n)
            emit4<SHIFT, SXOR, WU, WF, NT>(ou, of, base + o, n - o, v0, v1, v2, v3, sh);
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


// ------------------------------------------------ 64-bit indices, partitions ----
//
// Part p of 2^q receives the indices i = m 2^q + r, r = rev_q(p); the kernels enumerate m.
// For a digital sequence, bit k of m selects column k + q, and the bits of r select a fixed
// set of columns below q whose XOR is formed once per wavefront.  m has up to 64 bits, so
// the chunk part takes a reduction over the whole wavefront (lanes 8..63 select columns
// 8..63 of the subsequence), and a second one for chunk h + 1 when `first` is not a
// multiple of 256.

// XOR of v over all 64 lanes, as a wave-uniform value.
__device__ __forceinline__ uint32_t wave_xor(uint32_t v) {
    const uint32_t h = half_wave_xor(v);
    return __builtin_amdgcn_readlane(h, 31) ^ __builtin_amdgcn_readlane(h, 63);
}

// Needs first % 4 == 0, ld % 4 == 0, 16-byte aligned outputs, n <= 2^31 and every m below
// 2^(columns - q).
template <bool NUS, bool SHIFT, bool SXOR, bool WU, bool WF, bool NT>
__global__ __launch_bounds__(kWave) void sobol64_fast(const uint32_t* __restrict__ mats, uint32_t columns,
                                                      uint32_t q, uint32_t r, uint64_t first, uint32_t n,
                                                      const uint32_t* __restrict__ seeds,
                                                      const uint32_t* __restrict__ shifts, uint32_t* __restrict__ ou,
                                                      float* __restrict__ of, uint64_t ld, uint32_t cpw,
                                                      uint32_t nchunks) {
    dev::set_fp32_round_toward_zero();
    const uint32_t j = blockIdx.y;
    const uint32_t lane = threadIdx.x;
    const uint32_t cb = blockIdx.x * cpw;
    const uint32_t ce = min(cb + cpw, nchunks);
    const uint32_t* cj = mats + uint64_t(j) * columns;
    uint32_t col = lane + q < columns ? cj[lane + q] : 0u;               // image of bit `lane` of m
    uint32_t low = (lane < q && ((r >> lane) & 1u)) ? cj[lane] : 0u;     // bits of r
    if constexpr (NUS) {
        col = dev::brev(col);
        low = dev::brev(low);
    }
    const uint32_t xr = wave_xor(low);
    const uint32_t seed = NUS ? seeds[j] : 0u;
    const uint32_t sm = dev::seed_multiplier(seed);
    const uint32_t sh = SHIFT ? shifts[j] : 0u;
    const uint32_t t = (static_cast<uint32_t>(first) & 255u) + 4u * lane;
    const uint32_t carry = 0u - (t >> 8);
    const bool straddle = (first & 255u) != 0;
    uint32_t xlo = xr;
#pragma unroll
    for (int k = 2; k < 8; ++k) xlo ^= (0u - ((t >> k) & 1u)) & __builtin_amdgcn_readlane(col, k);
    const uint32_t col0 = __builtin_amdgcn_readlane(col, 0), col1 = __builtin_amdgcn_readlane(col, 1);
    const uint64_t hb = first >> 8;
    const uint64_t base = uint64_t(j) * ld;
    for (uint32_t c = cb; c < ce; ++c) {
        const uint64_t h = hb + c;
        const uint32_t sel = lane >= 8u ? static_cast<uint32_t>(h >> (lane - 8u)) & 1u : 0u;
        uint32_t x = wave_xor(sel ? col : 0u);
        if (straddle) {
            const uint32_t sel1 = lane >= 8u ? static_cast<uint32_t>((h + 1u) >> (lane - 8u)) & 1u : 0u;
            const uint32_t x1 = wave_xor(sel1 ? col : 0u);
            x ^= (x ^ x1) & carry;
        }
        x ^= xlo;
        uint32_t v0 = x, v1 = x ^ col0, v2 = x ^ col1, v3 = x ^ col0 ^ col1;
        if constexpr (NUS) {
            v0 = dev::nus_from_mirrored(v0, seed, sm);
            v1 = dev::nus_from_mirrored(v1, seed, sm);
            v2 = dev::nus_from_mirrored(v2, seed, sm);
            v3 = dev::nus_from_mirrored(v3, seed, sm);
        }
        const uint32_t o = c * kChunk + 4u * lane;
        if (o + 4u <= n)
            emit4<SHIFT, SXOR, WU, WF, NT>(ou, of, base + o, 4u, v0, v1, v2, v3, sh);
        else if (o < n)
            emit4<SHIFT, SXOR, WU, WF, NT>(ou, of, base + o, n - o, v0, v1, v2, v3, sh);
    }
}

struct Sobol64Lds {
    uint32_t cols[QMC_MAX_DIMS][64];
    uint32_t seed[QMC_MAX_DIMS];
    uint32_t sm[QMC_MAX_DIMS];
    uint32_t shift[QMC_MAX_DIMS];
};

// Any alignment: one index per thread, the plain product over all 64 index bits.
template <bool NUS, bool SHIFT, bool SXOR, bool WU, bool WF>
__global__ __launch_bounds__(kBlock) void sobol64_general(const uint32_t* __restrict__ mats, uint32_t columns,
                                                          uint32_t s, uint32_t q, uint32_t r, uint64_t first,
                                                          uint32_t n, const uint32_t* __restrict__ seeds,
                                                          const uint32_t* __restrict__ shifts,
                                                          uint32_t* __restrict__ ou, float* __restrict__ of,
                                                          uint64_t ld) {
    dev::set_fp32_round_toward_zero();
    __shared__ Sobol64Lds L;
    for (uint32_t t = threadIdx.x; t < s * 64; t += blockDim.x) {
        const uint32_t k = t & 63u;
        const uint32_t c = k < columns ? mats[uint64_t(t >> 6) * columns + k] : 0u;
        L.cols[t >> 6][k] = NUS ? dev::brev(c) : c;
    }
    for (uint32_t t = threadIdx.x; t < s; t += blockDim.x) {
        if constexpr (NUS) {
            L.seed[t] = seeds[t];
            L.sm[t] = dev::seed_multiplier(seeds[t]);
        }
        if constexpr (SHIFT) L.shift[t] = shifts[t];
    }
    __syncthreads();
    for (uint32_t o = blockIdx.x * kBlock + threadIdx.x; o < n; o += gridDim.x * kBlock) {
        const uint64_t i = ((first + o) << q) | r;
        const uint32_t ilo = static_cast<uint32_t>(i), ihi = static_cast<uint32_t>(i >> 32);
        for (uint32_t j = 0; j < s; ++j) {
            uint32_t v = matrix_product(L.cols[j], ilo) ^ matrix_product(L.cols[j] + 32, ihi);
            if constexpr (NUS) v = dev::nus_from_mirrored(v, L.seed[j], L.sm[j]);
            if constexpr (SHIFT) v = dev::apply_shift<SXOR>(v, L.shift[j]);
            if constexpr (WU) ou[uint64_t(j) * ld + o] = v;
            if constexpr (WF) of[uint64_t(j) * ld + o] = dev::u32_to_unifloat_rtz(v);
        }
    }
}

// floor(2^32 frac(phi_2(i) g)) for a 64-bit index: brev64(i) = brev(ilo) 2^32 + brev(ihi), and
// the top word of its product with g modulo 2^64 is brev(ilo) g + high word of brev(ihi) g.
__device__ __forceinline__ uint32_t lattice64_value(uint64_t i, uint32_t g) {
    const uint32_t hi = dev::brev(static_cast<uint32_t>(i)), lo = dev::brev(static_cast<uint32_t>(i >> 32));
    return hi * g + __umulhi(lo, g);
}

template <bool BACK, bool SHIFT, bool SXOR, bool WU, bool WF, bool NT>
__global__ __launch_bounds__(kWave) void lattice64_fast(const uint32_t* __restrict__ gen, uint32_t q, uint32_t r,
                                                        uint64_t first, uint32_t n,
                                                        const uint32_t* __restrict__ shifts,
                                                        uint32_t* __restrict__ ou, float* __restrict__ of, uint64_t ld,
                                                        uint32_t cpw, uint32_t nchunks) {
    dev::set_fp32_round_toward_zero();
    const uint32_t j = blockIdx.y;
    const uint32_t lane = threadIdx.x;
    const uint32_t cb = blockIdx.x * cpw;
    const uint32_t ce = min(cb + cpw, nchunks);
    const uint32_t g = gen[j];
    const uint32_t sh = SHIFT ? shifts[j] : 0u;
    const uint64_t base = uint64_t(j) * ld;
    const uint64_t flip = BACK ? ~uint64_t(0) : 0u;
    for (uint32_t c = cb; c < ce; ++c) {
        const uint32_t o = c * kChunk + 4u * lane;
        const uint64_t m = first + o;
        const uint32_t v0 = lattice64_value(((m << q) | r) ^ flip, g);
        const uint32_t v1 = lattice64_value((((m + 1u) << q) | r) ^ flip, g);
        const uint32_t v2 = lattice64_value((((m + 2u) << q) | r) ^ flip, g);
        const uint32_t v3 = lattice64_value((((m + 3u) << q) | r) ^ flip, g);
        if (o + 4u <= n)
            emit4<SHIFT, SXOR, WU, WF, NT>(ou, of, base + o, 4u, v0, v1, v2, v3, sh);
        else if (o < n)
            emit4<SHIFT, SXOR, WU, WF, NT>(ou, of, base + o, n - o, v0, v1, v2, v3, sh);
    }
}

template <bool BACK, bool SHIFT, bool SXOR, bool WU, bool WF>
__global__ __launch_bounds__(kBlock) void lattice64_general(const uint32_t* __restrict__ gen, uint32_t s, uint32_t q,
                                                            uint32_t r, uint64_t first, uint32_t n,
                                                            const uint32_t* __restrict__ shifts,
                                                            uint32_t* __restrict__ ou, float* __restrict__ of,
                                                            uint64_t ld) {
    dev::set_fp32_round_toward_zero();
    __shared__ LatticeLds L;
    stage_lattice<SHIFT>(L, gen, s, shifts);
    for (uint32_t o = blockIdx.x * kBlock + threadIdx.x; o < n; o += gridDim.x * kBlock) {
        const uint64_t i = (((first + o) << q) | r) ^ (BACK ? ~uint64_t(0) : 0u);
        for (uint32_t j = 0; j < s; ++j) {
            uint32_t v = lattice64_value(i, L.g[j]);
            if constexpr (SHIFT) v = dev::apply_shift<SXOR>(v, L.shift[j]);
            if constexpr (WU) ou[uint64_t(j) * ld + o] = v;
            if constexpr (WF) of[uint64_t(j) * ld + o] = dev::u32_to_unifloat_rtz(v);
        }
    }
}

// ------------------------------------------------------------ point-major ----
//
// out[(i - first) * ld + j]: a wavefront takes 64 consecutive points, forms up to 32
// components of its lane's point into an LDS tile, then writes the tile (eight rows of 128 bytes
// per 16-byte store instruction when rows are 16-byte aligned, else two rows of 4-byte stores),
// and repeats for the next 32 dimensions.  Blocks of four
// wavefronts share the staged matrices, so the LDS a wavefront needs stays small and more of
// them stream at once.

constexpr uint32_t kPmWaves = 4;  // wavefronts per block
// Blocks launched per compute unit (each wavefront then takes about four tiles at 2^24 points):
// 2^24 x 32 Sobol' points took 0.82 ms with 8 per compute unit, 0.79 with 16, 0.77 with 32,
// 0.74 with 64 and 0.91 with one tile per wavefront, where staging the matrices dominates.
constexpr uint32_t kPmBlocksPerCu = 64;

// Writes the wavefront's tile (rows < rows, components j0 .. j0 + sg) to the outputs.  V16 (rows
// of 16-byte aligned components, sg = 32): a lane stores components 4 (lane mod 8) .. + 3 of row
// lane / 8 as one 16-byte store, eight rows per instruction; otherwise two rows of 4-byte stores.
template <bool WU, bool WF, bool V16>
__device__ __forceinline__ void store_tile(const uint32_t (&tile)[kWave][33], uint32_t lane, uint32_t rows,
                                           uint32_t sg, uint32_t o0, uint32_t j0, uint32_t* __restrict__ ou,
                                           float* __restrict__ of, uint64_t ld) {
    if (V16 && sg == 32) {
        const uint32_t c = (lane & 7u) * 4u;
#pragma unroll 2
        for (uint32_t r0 = 0; r0 < rows; r0 += 8) {
            const uint32_t r = r0 + (lane >> 3);
            if (r < rows) {
                const u32x4 v{tile[r][c], tile[r][c + 1], tile[r][c + 2], tile[r][c + 3]};
                const uint64_t at = uint64_t(o0 + r) * ld + j0 + c;
                if constexpr (WU) *reinterpret_cast<u32x4*>(ou + at) = v;
                if constexpr (WF)
                    *reinterpret_cast<f32x4*>(of + at) =
                        f32x4{dev::u32_to_unifloat_rtz(v.x), dev::u32_to_unifloat_rtz(v.y),
                              dev::u32_to_unifloat_rtz(v.z), dev::u32_to_unifloat_rtz(v.w)};
            }
        }
        return;
    }
    const uint32_t k32 = lane & 31u, sub = lane >> 5;
#pragma unroll 4
    for (uint32_t r0 = 0; r0 < rows; r0 += 2) {
        const uint32_t r = r0 + sub;
        if (k32 < sg && r < rows) {
            const uint32_t v = tile[r][k32];
            const uint64_t at = uint64_t(o0 + r) * ld + j0 + k32;
            if constexpr (WU) ou[at] = v;
            if constexpr (WF) of[at] = dev::u32_to_unifloat_rtz(v);
        }
    }
}

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The point of index i = 64 h + lane (first a multiple of 64) is the XOR of a part from the
// high index bits, the same for the whole wavefront (lanes 6..31 select a column each, XOR
// reduction in DPP), and a part from the lane's six low bits, tabulated per dimension and lane
// once per block; other starts use the plain matrix product.  SM: dimensions the block stages
// (32 or 64).
template <int SM, bool NUS, bool SHIFT, bool SXOR, bool WU, bool WF, bool SPLIT, bool V16>
__global__ __launch_bounds__(kWave * kPmWaves) void sobol_point_major(const uint32_t* __restrict__ mats, uint32_t s,
                                                                      uint32_t first, uint32_t n,
                                                                      const uint32_t* __restrict__ seeds,
                                                                      const uint32_t* __restrict__ shifts,
                                                                      uint32_t* __restrict__ ou, float* __restrict__ of,
                                                                      uint64_t ld) {
    dev::set_fp32_round_toward_zero();
    __shared__ uint32_t cols[SM][32];
    __shared__ uint32_t seed[SM], smul[SM], shift[SM];
    __shared__ uint32_t lo[SPLIT ? SM : 1][kWave];
    __shared__ uint32_t tiles[kPmWaves][kWave][33];
    for (uint32_t t = threadIdx.x; t < s * 32; t += blockDim.x) {
        const uint32_t c = mats[t];
        cols[t >> 5][t & 31] = NUS ? dev::brev(c) : c;
    }
    for (uint32_t t = threadIdx.x; t < s; t += blockDim.x) {
        if constexpr (NUS) {
            seed[t] = seeds[t];
            smul[t] = dev::seed_multiplier(seeds[t]);
        }
        if constexpr (SHIFT) shift[t] = shifts[t];
    }
    __syncthreads();
    if constexpr (SPLIT) {
        for (uint32_t t = threadIdx.x; t < s * kWave; t += blockDim.x) {
            const uint32_t j = t / kWave, l = t % kWave;
            uint32_t x = 0;
#pragma unroll
            for (int k = 0; k < 6; ++k) x ^= (0u - ((l >> k) & 1u)) & cols[j][k];
            lo[j][l] = x;
        }
        __syncthreads();
    }
    const uint32_t wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const uint32_t k32 = lane & 31u;
    uint32_t(&tile)[kWave][33] = tiles[wave];
    // wavefronts run different numbers of tiles: only wavefront-level synchronisation below
    for (uint32_t o0 = (blockIdx.x * kPmWaves + wave) * kWave; o0 < n; o0 += gridDim.x * kPmWaves * kWave) {
        const uint32_t i = first + o0 + lane;
        const uint32_t h = (first + o0) >> 6;
        const uint32_t rows = min(n - o0, kWave);
        for (uint32_t j0 = 0; j0 < s; j0 += 32) {
            const uint32_t sg = min(s - j0, 32u);
#pragma unroll 4
            for (uint32_t jj = 0; jj < sg; ++jj) {
                const uint32_t j = j0 + jj;
                uint32_t v;
                if constexpr (SPLIT) {
                    const uint32_t part = half_wave_xor((k32 >= 6u && ((h >> (k32 - 6u)) & 1u)) ? cols[j][k32] : 0u);
                    v = __builtin_amdgcn_readlane(part, 31) ^ lo[j][lane];
                } else {
                    v = matrix_product(cols[j], i);
                }
                if constexpr (NUS) v = dev::nus_from_mirrored(v, seed[j], smul[j]);
                if constexpr (SHIFT) v = dev::apply_shift<SXOR>(v, shift[j]);
                tile[lane][jj] = v;
            }
            wave_sync();
            store_tile<WU, WF, V16>(tile, lane, rows, sg, o0, j0, ou, of, ld);
            wave_sync();
        }
    }
}

// Lattice points in the same tiles: a lane forms brev(i) once and multiplies it by each
// component of the generator (Alg. 4).
template <bool BACK, bool SHIFT, bool SXOR, bool WU, bool WF, bool V16>
__global__ __launch_bounds__(kWave * kPmWaves) void lattice_point_major(const uint32_t* __restrict__ gen, uint32_t s,
                                                                        uint32_t first, uint32_t n,
                                                                        const uint32_t* __restrict__ shifts,
                                                                        uint32_t* __restrict__ ou,
                                                                        float* __restrict__ of, uint64_t ld) {
    dev::set_fp32_round_toward_zero();
    __shared__ LatticeLds L;
    __shared__ uint32_t tiles[kPmWaves][kWave][33];
    stage_lattice<SHIFT>(L, gen, s, shifts);
    const uint32_t wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const uint32_t k32 = lane & 31u;
    uint32_t(&tile)[kWave][33] = tiles[wave];
    for (uint32_t o0 = (blockIdx.x * kPmWaves + wave) * kWave; o0 < n; o0 += gridDim.x * kPmWaves * kWave) {
        const uint32_t i = first + o0 + lane;
        const uint32_t b = dev::brev(BACK ? ~i : i);
        const uint32_t rows = min(n - o0, kWave);
        for (uint32_t j0 = 0; j0 < s; j0 += 32) {
            const uint32_t sg = min(s - j0, 32u);
#pragma unroll 4
            for (uint32_t jj = 0; jj < sg; ++jj) {
                uint32_t v = b * L.g[j0 + jj];
                if constexpr (SHIFT) v = dev::apply_shift<SXOR>(v, L.shift[j0 + jj]);
                tile[lane][jj] = v;
            }
            wave_sync();
            store_tile<WU, WF, V16>(tile, lane, rows, sg, o0, j0, ou, of, ld);
            wave_sync();
        }
    }
}

// ------------------------------------------------------------------ Halton ----
//
// Radical inversion in prime bases (Sec. 2.2): component j of point i is
// floor(2^32 phi_{b,sigma}(i mod b^M)) with b the j-th prime and b^M the largest power of b in
// 32 bits.  With all M digits formed (leading zeros included; sigma(0) = 0 for every
// permutation used), phi = R / b^M for the mirrored digit integer R, so one exact division
// by a per-dimension constant ends the loop.  Digits come from a multiply by floor(2^32 / b)
// and one correction step; base 2 is the bit reversal of the reduced index.

__constant__ uint32_t kPrimes[QMC_MAX_DIMS] = {
    2,   3,   5,   7,   11,  13,  17,  19,  23,  29,  31,  37,  41,  43,  47,  53,  59,  61,  67,  71,  73,  79,
    83,  89,  97,  101, 103, 107, 109, 113, 127, 131, 137, 139, 149, 151, 157, 163, 167, 173, 179, 181, 191, 193,
    197, 199, 211, 223, 227, 229, 233, 239, 241, 251, 257, 263, 269, 271, 277, 281, 283, 293, 307, 311};

constexpr uint32_t kMaxBase = 311;

struct HaltonBase {
    uint32_t b, digits, maxpow, rcp;
    uint32_t zero2;  // base 2 with an even linear factor: sigma = (0, 0), every value is 0
    double inv_maxpow, scale;
};

__device__ __forceinline__ HaltonBase halton_base(uint32_t b) {
    HaltonBase h;
    h.b = b;
    uint64_t q = b;
    uint32_t m = 1;
    while (q * b <= 0xFFFFFFFFull) {
        q *= b;
        ++m;
    }
    h.digits = m;
    h.maxpow = static_cast<uint32_t>(q);
    h.rcp = static_cast<uint32_t>((uint64_t(1) << 32) / b);
    h.inv_maxpow = 1.0 / static_cast<double>(q);
    h.scale = 4294967296.0 / static_cast<double>(q);
    h.zero2 = 0;
    return h;
}

// Faure's permutations of the first QMC_MAX_DIMS primes, one after another, formed at compile
// time: sigma_2 = (0, 1); for even y, 2 sigma_{y/2} followed by 2 sigma_{y/2} + 1; for odd y,
// sigma_{y-1} with every value >= (y-1)/2 raised by one and (y-1)/2 inserted in the middle.
constexpr uint32_t kPrimeList[QMC_MAX_DIMS] = {
    2,   3,   5,   7,   11,  13,  17,  19,  23,  29,  31,  37,  41,  43,  47,  53,  59,  61,  67,  71,  73,  79,
    83,  89,  97,  101, 103, 107, 109, 113, 127, 131, 137, 139, 149, 151, 157, 163, 167, 173, 179, 181, 191, 193,
    197, 199, 211, 223, 227, 229, 233, 239, 241, 251, 257, 263, 269, 271, 277, 281, 283, 293, 307, 311};

constexpr uint32_t faure_total() {
    uint32_t t = 0;
    for (uint32_t j = 0; j < QMC_MAX_DIMS; ++j) t += kPrimeList[j];
    return t;
}

struct FaureTable {
    uint16_t v[faure_total()];
    uint16_t off[QMC_MAX_DIMS];  // start of base j's permutation in v
};

struct FaureAll {  // sigma_y for every y <= kMaxBase (compile-time scratch)
    uint16_t p[kMaxBase + 1][kMaxBase + 1];
};

constexpr FaureTable make_faure_table() {
    FaureAll all{};
    all.p[2][1] = 1;
    for (uint32_t y = 3; y <= kMaxBase; ++y) {
        if (y % 2 == 0) {
            const uint32_t h = y / 2;
            for (uint32_t a = 0; a < h; ++a) {
                all.p[y][a] = static_cast<uint16_t>(2 * all.p[h][a]);
                all.p[y][a + h] = static_cast<uint16_t>(2 * all.p[h][a] + 1);
            }
        } else {
            const uint32_t c = (y - 1) / 2;
            for (uint32_t a = 0; a < y; ++a) {
                if (a == c) {
                    all.p[y][a] = static_cast<uint16_t>(c);
                } else {
                    const uint32_t t = all.p[y - 1][a < c ? a : a - 1];
                    all.p[y][a] = static_cast<uint16_t>(t >= c ? t + 1 : t);
                }
            }
        }
    }
    FaureTable t{};
    uint32_t pos = 0;
    for (uint32_t j = 0; j < QMC_MAX_DIMS; ++j) {
        const uint32_t b = kPrimeList[j];
        t.off[j] = static_cast<uint16_t>(pos);
        for (uint32_t a = 0; a < b; ++a) t.v[pos++] = all.p[b][a];
    }
    return t;
}

__constant__ FaureTable kFaure = make_faure_table();

// Digit permutation of dimension j (base b) into LDS (one wavefront).  MODE 1: Faure's
// permutation, copied from the compile-time table; MODE 2: sigma(a) = f a mod b.  Returns the
// buffer that holds it.
template <uint32_t MODE>
__device__ uint32_t* build_permutation(uint32_t b, uint32_t f, uint32_t j, uint32_t (&buf)[2][kMaxBase + 1]) {
    const uint32_t lane = threadIdx.x;
    if constexpr (MODE == 2) {
        for (uint32_t a = lane; a < b; a += kWave) buf[0][a] = static_cast<uint32_t>((uint64_t(f) * a) % b);
    } else {
        const uint32_t off = kFaure.off[j];
        for (uint32_t a = lane; a < b; a += kWave) buf[0][a] = kFaure.v[off + a];
    }
    __syncthreads();
    return buf[0];
}

// floor(2^32 phi_{b,sigma}(i mod b^M)) for b >= 3.
template <uint32_t MODE>
__device__ __forceinline__ uint32_t halton_component(uint32_t i, const HaltonBase& h, const uint32_t* sig) {
    uint32_t q = static_cast<uint32_t>(static_cast<double>(i) * h.inv_maxpow);
    uint64_t t = uint64_t(q) * h.maxpow;
    if (t > i) {  // the estimate can be one too high or too low
        --q;
        t -= h.maxpow;
    } else if (i - t >= h.maxpow) {
        ++q;
        t += h.maxpow;
    }
    uint32_t x = static_cast<uint32_t>(i - t);
    uint32_t r = 0;
    for (uint32_t k = 0; k < h.digits; ++k) {
        uint32_t qq = __umulhi(x, h.rcp);
        uint32_t d = x - qq * h.b;
        if (d >= h.b) {
            ++qq;
            d -= h.b;
        }
        r = r * h.b + (MODE == 0 ? d : sig[d]);
        x = qq;
    }
    uint32_t v = static_cast<uint32_t>(static_cast<double>(r) * h.scale);
    const uint64_t num = uint64_t(r) << 32;
    const uint64_t den = uint64_t(v) * h.maxpow;
    if (den > num)
        --v;
    else if (num - den >= h.maxpow)
        ++v;
    return v;
}

template <uint32_t MODE>
__device__ __forceinline__ uint32_t halton_value(uint32_t i, const HaltonBase& h, const uint32_t* sig) {
    if (h.b == 2) return h.zero2 ? 0u : dev::brev(i & 0x7FFFFFFFu);
    return halton_component<MODE>(i, h, sig);
}

// Per-dimension constants of the table-driven Halton kernel, computed on the host.  With
// x = i mod b^M split as x = hi b^e + lo (lo: the e low digits), phi = R_e(lo) / b^e + H(hi) / b^M,
// R_e the mirrored e-digit value and H the mirrored value of the M - e high digits (weights
// b^(M-e-1) down to 1).  Both terms are kept as 64-bit fractions floor(2^64 .):
//   flo[lo] = floor(2^64 R_e(lo) / b^e) = R_e(lo) qe + floor(R_e(lo) re / b^e),
//   fhi(hi) = floor(2^64 H(hi) / b^M)   = H qm + floor(H rm / b^M),
// with 2^64 = qe b^e + re = qm b^M + rm.  Their sum S satisfies S <= 2^64 phi < S + 2, so
// floor(2^32 phi) is the high word of S unless its low word is 2^32 - 2 or 2^32 - 1 (then the
// exact digit loop decides).  The table size b^e is chosen so that the high parts of a
// wavefront's indices (`run` chunks of 256) span at most 64 consecutive values, one per lane:
// b^e >= 17 for 4 chunks, b^e >= 34 for 8.
struct HaltonDim {
    uint64_t qm, qe;
    uint32_t rm, re;
    uint32_t e, le;      // low digits per table entry and b^e
    uint32_t le_magic;   // ceil(2^32 / b^e): exact quotients of y < 2^32 / b^e
    double inv_maxpow;   // 1 / b^M (estimate for floor(H rm / b^M))
};
struct HaltonTable {
    HaltonDim d[QMC_MAX_DIMS];
};

constexpr uint32_t kHaltonMaxLow = 961;  // largest b^e (b = 31, e = 2, runs of 8 chunks)

// Mirrored value of the `digits` low base-b digits of x (the lowest becomes the most significant).
template <uint32_t MODE>
__device__ __forceinline__ uint32_t mirrored_digits(uint32_t x, uint32_t digits, const HaltonBase& h,
                                                    const uint32_t* sig) {
    uint32_t r = 0;
    for (uint32_t k = 0; k < digits; ++k) {
        uint32_t qq = __umulhi(x, h.rcp);
        uint32_t d = x - qq * h.b;
        if (d >= h.b) {
            ++qq;
            d -= h.b;
        }
        r = r * h.b + (MODE == 0 ? d : sig[d]);
        x = qq;
    }
    return r;
}

// Block (x, j): dimension j, chunks [x * run, (x + 1) * run) of 256 indices, four consecutive
// indices per lane (first % 4 == 0, ld % 4 == 0, 16-byte aligned outputs); the table was made
// for this run length.
template <uint32_t MODE, bool WU, bool WF, bool NT>
__global__ __launch_bounds__(kWave) void halton_fast(uint32_t first, uint32_t n, const uint32_t* __restrict__ factors,
                                                     uint32_t* __restrict__ ou, float* __restrict__ of, uint64_t ld,
                                                     uint32_t run, uint32_t nchunks, HaltonTable tab) {
    dev::set_fp32_round_toward_zero();
    __shared__ uint32_t buf[2][kMaxBase + 1];
    __shared__ uint64_t flo[kHaltonMaxLow];
    __shared__ uint64_t fhi[kWave];
    const uint32_t j = blockIdx.y;
    HaltonBase h = halton_base(kPrimes[j]);
    const uint32_t f = MODE == 2 ? factors[j] : 1u;
    if (MODE == 2 && h.b == 2) h.zero2 = (f & 1u) ? 0u : 1u;
    const uint32_t* sig = nullptr;
    if constexpr (MODE != 0) sig = build_permutation<MODE>(h.b, f, j, buf);
    const uint32_t lane = threadIdx.x;
    const uint32_t cb = blockIdx.x * run;
    const uint32_t ce = min(cb + run, nchunks);
    const uint64_t base = uint64_t(j) * ld;
    const uint32_t i0 = first + cb * kChunk;                 // first index of the wavefront
    const uint32_t x0 = i0 % h.maxpow;                        // its reduced index
    const uint32_t span = (ce - cb) * kChunk;
    if (h.b == 2 || uint64_t(x0) + span > h.maxpow) {
        // base 2, or the reduction wraps inside this wavefront's range: digit loop per index
        for (uint32_t c = cb; c < ce; ++c) {
            const uint32_t o = c * kChunk + 4u * lane;
            const uint32_t i = first + o;
            const uint32_t v0 = halton_value<MODE>(i, h, sig), v1 = halton_value<MODE>(i + 1u, h, sig);
            const uint32_t v2 = halton_value<MODE>(i + 2u, h, sig), v3 = halton_value<MODE>(i + 3u, h, sig);
            if (o + 4u <= n)
                emit4<false, false, WU, WF, NT>(ou, of, base + o, 4u, v0, v1, v2, v3, 0u);
            else if (o < n)
                emit4<false, false, WU, WF, NT>(ou, of, base + o, n - o, v0, v1, v2, v3, 0u);
        }
        return;
    }
    const HaltonDim& hd = tab.d[j];
    for (uint32_t t = lane; t < hd.le; t += kWave) {
        const uint32_t r = mirrored_digits<MODE>(t, hd.e, h, sig);
        flo[t] = uint64_t(r) * hd.qe + (r * hd.re) / hd.le;
    }
    // lane l: the high part hi = x0 / b^e + l
    const uint32_t hw0 = x0 / hd.le;
    {
        const uint32_t H = mirrored_digits<MODE>(hw0 + lane, h.digits - hd.e, h, sig);
        const uint64_t N = uint64_t(H) * hd.rm;
        int64_t q = static_cast<int64_t>(static_cast<double>(N) * hd.inv_maxpow);
        int64_t rem = static_cast<int64_t>(N - uint64_t(q) * h.maxpow);
#pragma unroll
        for (int t = 0; t < 3; ++t) {
            if (rem < 0) {
                --q;
                rem += h.maxpow;
            } else if (rem >= int64_t(h.maxpow)) {
                ++q;
                rem -= h.maxpow;
            }
        }
        fhi[lane] = uint64_t(H) * hd.qm + uint64_t(q);
    }
    __syncthreads();
    const uint32_t y0 = x0 - hw0 * hd.le;  // offset of index i0 above hw0 b^e (below b^e)
    for (uint32_t c = cb; c < ce; ++c) {
        const uint32_t o = c * kChunk + 4u * lane;
        uint32_t v[4];
#pragma unroll
        for (uint32_t k = 0; k < 4; ++k) {
            const uint32_t y = y0 + (o - cb * kChunk) + k;
            const uint32_t dl = __umulhi(y, hd.le_magic);
            const uint32_t lo = y - dl * hd.le;
            const uint64_t S = flo[lo] + fhi[dl];
            v[k] = static_cast<uint32_t>(S >> 32);
            if (static_cast<uint32_t>(S) >= 0xFFFFFFFEu) v[k] = halton_component<MODE>(first + o + k, h, sig);
        }
        if (o + 4u <= n)
            emit4<false, false, WU, WF, NT>(ou, of, base + o, 4u, v[0], v[1], v[2], v[3], 0u);
        else if (o < n)
            emit4<false, false, WU, WF, NT>(ou, of, base + o, n - o, v[0], v[1], v[2], v[3], 0u);
    }
}

// Any alignment: block (x, j) covers indices x * 64 + lane + k * 64 * gridDim.x of dimension j.
template <uint32_t MODE, bool WU, bool WF>
__global__ __launch_bounds__(kWave) void halton_general(uint32_t first, uint32_t n,
                                                        const uint32_t* __restrict__ factors,
                                                        uint32_t* __restrict__ ou, float* __restrict__ of,
                                                        uint64_t ld) {
    dev::set_fp32_round_toward_zero();
    __shared__ uint32_t buf[2][kMaxBase + 1];
    const uint32_t j = blockIdx.y;
    HaltonBase h = halton_base(kPrimes[j]);
    const uint32_t f = MODE == 2 ? factors[j] : 1u;
    if (MODE == 2 && h.b == 2) h.zero2 = (f & 1u) ? 0u : 1u;
    const uint32_t* sig = nullptr;
    if constexpr (MODE != 0) sig = build_permutation<MODE>(h.b, f, j, buf);
    for (uint32_t o = blockIdx.x * kWave + threadIdx.x; o < n; o += gridDim.x * kWave) {
        const uint32_t v = halton_value<MODE>(first + o, h, sig);
        if constexpr (WU) ou[uint64_t(j) * ld + o] = v;
        if constexpr (WF) of[uint64_t(j) * ld + o] = dev::u32_to_unifloat_rtz(v);
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

// first + n <= 2^bits (bits <= 64).
bool index_range_ok(uint64_t first, uint64_t n, uint32_t bits) {
    if (bits >= 64) return n == 0 || n - 1 <= ~first;
    const uint64_t lim = uint64_t(1) << bits;
    return first <= lim && n <= lim - first;
}

// Shared validation of the generation calls.
qmc_status validate_generation(const char* who, qmc_context ctx, const void* table, uint64_t table_bytes_per_dim,
                               uint32_t s, uint64_t first, uint64_t n, uint32_t flags, uint32_t allowed_flags,
                               const void* aux0, const void* aux1, const uint32_t* ou, const float* of, uint64_t ld,
                               uint32_t index_bits = 32) {
    if (!ctx) return fail(QMC_ERR_INVALID_ARGUMENT, "%s: context is NULL", who);
    if (s == 0 || s > QMC_MAX_DIMS) return fail(QMC_ERR_OUT_OF_RANGE, "%s: s = %u outside [1, %d]", who, s, QMC_MAX_DIMS);
    if (!index_range_ok(first, n, index_bits))
        return fail(QMC_ERR_OUT_OF_RANGE, "%s: first + n exceeds 2^%u (first=%llu n=%llu)", who, index_bits,
                    (unsigned long long)first, (unsigned long long)n);
    if (flags & ~allowed_flags) return fail(QMC_ERR_INVALID_ARGUMENT, "%s: unknown flags 0x%x", who, flags);
    if (n == 0) return QMC_OK;
    if (!table) return fail(QMC_ERR_INVALID_ARGUMENT, "%s: table pointer is NULL", who);
    if (!ou && !of) return fail(QMC_ERR_INVALID_ARGUMENT, "%s: both outputs are NULL", who);
    const bool pm = (flags & QMC_POINT_MAJOR) != 0;
    if (!pm && ld < n)
        return fail(QMC_ERR_INVALID_ARGUMENT, "%s: ld (%llu) < n (%llu)", who, (unsigned long long)ld,
                    (unsigned long long)n);
    if (pm && ld < s)
        return fail(QMC_ERR_INVALID_ARGUMENT, "%s: point-major ld (%llu) < s (%u)", who, (unsigned long long)ld, s);
    if (ld > (uint64_t(1) << 56) / (pm ? n : s)) return fail(QMC_ERR_OUT_OF_RANGE, "%s: ld too large", who);
    if (!pm && n > (uint64_t(1) << 56)) return fail(QMC_ERR_OUT_OF_RANGE, "%s: n too large", who);
    const uint64_t out_bytes = (pm ? (n - 1) * ld + s : (uint64_t(s) - 1) * ld + n) * 4;
    if (ranges_overlap(ou, out_bytes, of, out_bytes))
        return fail(QMC_ERR_INVALID_ARGUMENT, "%s: outputs overlap", who);
    const void* ins[3] = {table, aux0, aux1};
    const uint64_t in_bytes[3] = {uint64_t(s) * table_bytes_per_dim, uint64_t(s) * 4, uint64_t(s) * 4};
    for (int k = 0; k < 3; ++k)
        if (ranges_overlap(ins[k], in_bytes[k], ou, out_bytes) || ranges_overlap(ins[k], in_bytes[k], of, out_bytes))
            return fail(QMC_ERR_INVALID_ARGUMENT, "%s: an output overlaps an input", who);
    return QMC_OK;
}

// Constants of halton_fast for the first s primes and runs of `run` chunks (see HaltonDim).
void halton_table(uint32_t s, uint32_t run, HaltonTable* t) {
    const uint64_t min_le = (uint64_t(kChunk) * run - 1) / 62 + 1;  // high parts span <= 64 values
    const unsigned __int128 two64 = static_cast<unsigned __int128>(1) << 64;
    for (uint32_t j = 0; j < s; ++j) {
        const uint64_t b = kPrimeList[j];
        uint64_t maxpow = b;
        while (maxpow * b <= 0xFFFFFFFFull) maxpow *= b;
        uint32_t e = 1;
        uint64_t le = b;
        while (le < min_le) {
            le *= b;
            ++e;
        }
        HaltonDim& d = t->d[j];
        d.qm = static_cast<uint64_t>(two64 / maxpow);
        d.rm = static_cast<uint32_t>(two64 % maxpow);
        d.qe = static_cast<uint64_t>(two64 / le);
        d.re = static_cast<uint32_t>(two64 % le);
        d.e = e;
        d.le = static_cast<uint32_t>(le);
        d.le_magic = static_cast<uint32_t>(((uint64_t(1) << 32) + le - 1) / le);
        d.inv_maxpow = 1.0 / static_cast<double>(maxpow);
    }
}

// The tuned launch shape is for both outputs (2 KiB per chunk of 256 indices).  With one output
// a chunk writes half as much, and one chunk per wavefront leaves the dispatch of wavefronts,
// not HBM, as the limit: such launches take four times as many chunks per wavefront.
GenTune launch_tune(GenTune tn, bool both_outputs) {
    if (!both_outputs) tn.chunks_per_wave *= 4;
    return tn;
}

// Grid of the fast kernels: x = runs of cpw chunks, y = dimension (dimension-major dispatch).
dim3 fast_grid(uint64_t n, uint32_t s, const GenTune& tn, uint32_t* nchunks) {
    *nchunks = static_cast<uint32_t>((n + kChunk - 1) / kChunk);
    const uint32_t cpw = tn.chunks_per_wave;
    return dim3((*nchunks + cpw - 1) / cpw, s);
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
    qmc_status st = validate_generation(who, ctx, matrices, 128, s, first, n, flags, QMC_SHIFT_XOR | QMC_POINT_MAJOR,
                                        nus_seeds, shifts, out_u32, out_f32, ld);
    if (st != QMC_OK || n == 0) return st;
    const bool pm = (flags & QMC_POINT_MAJOR) != 0;
    if (n > (uint64_t(1) << 31)) {  // kernels count indices in 32 bits: split [0, 2^32)
        const uint64_t h = uint64_t(1) << 31, step = pm ? h * ld : h;
        st = qmc_generate_sobol(ctx, stream, matrices, s, first, h, nus_seeds, shifts, flags, out_u32, out_f32, ld);
        if (st != QMC_OK) return st;
        return qmc_generate_sobol(ctx, stream, matrices, s, first + h, n - h, nus_seeds, shifts, flags,
                                  out_u32 ? out_u32 + step : nullptr, out_f32 ? out_f32 + step : nullptr, ld);
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
                    if (pm) {
                        const uint64_t want = (n + kWave * kPmWaves - 1) / (kWave * kPmWaves);
                        const uint32_t gx =
                            static_cast<uint32_t>(std::min<uint64_t>(want, uint64_t(ctx->num_cus) * kPmBlocksPerCu));
                        const bool v16 = (ld % 4 == 0) && aligned16(out_u32) && aligned16(out_f32);
                        with_bool(first % kWave == 0, [&](auto SPLIT) {
                            auto go = [&](auto SMV) {
                                with_bool(v16, [&](auto V16) {
                                    hipLaunchKernelGGL((sobol_point_major<decltype(SMV)::value, NUS.value, SH.value,
                                                                         SX.value, WU.value, WF.value, SPLIT.value,
                                                                         V16.value>),
                                                       dim3(gx), dim3(kWave * kPmWaves), 0, hs, matrices, s, first32,
                                                       nn, nus_seeds, shifts, out_u32, out_f32, ld);
                                });
                            };
                            if (s <= 32)
                                go(std::integral_constant<int, 32>{});
                            else
                                go(std::integral_constant<int, QMC_MAX_DIMS>{});
                        });
                    } else if (fast) {
                        with_bool(ctx->sobol_tune.nontemporal != 0, [&](auto NT) {
                            uint32_t nchunks;
                            const GenTune tn = launch_tune(ctx->sobol_tune, WU.value && WF.value);
                            const dim3 grid = fast_grid(nn, s, tn, &nchunks);
                            hipLaunchKernelGGL((sobol_fast<NUS.value, SH.value, SX.value, WU.value, WF.value, NT.value>),
                                               grid, dim3(kWave), 0, hs, matrices, first32, nn, nus_seeds, shifts,
                                               out_u32, out_f32, ld, tn.chunks_per_wave, nchunks);
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
                                        QMC_SHIFT_XOR | QMC_LATTICE_BACKWARD | QMC_POINT_MAJOR, shifts, nullptr,
                                        out_u32, out_f32, ld);
    if (st != QMC_OK || n == 0) return st;
    const bool pm = (flags & QMC_POINT_MAJOR) != 0;
    if (n > (uint64_t(1) << 31)) {  // kernels count indices in 32 bits: split [0, 2^32)
        const uint64_t h = uint64_t(1) << 31, step = pm ? h * ld : h;
        st = qmc_generate_lattice(ctx, stream, generator, s, first, h, shifts, flags, out_u32, out_f32, ld);
        if (st != QMC_OK) return st;
        return qmc_generate_lattice(ctx, stream, generator, s, first + h, n - h, shifts, flags,
                                    out_u32 ? out_u32 + step : nullptr, out_f32 ? out_f32 + step : nullptr, ld);
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
                    if (pm) {
                        const uint64_t want = (n + kWave * kPmWaves - 1) / (kWave * kPmWaves);
                        const uint32_t gx =
                            static_cast<uint32_t>(std::min<uint64_t>(want, uint64_t(ctx->num_cus) * kPmBlocksPerCu));
                        const bool v16 = (ld % 4 == 0) && aligned16(out_u32) && aligned16(out_f32);
                        with_bool(v16, [&](auto V16) {
                            hipLaunchKernelGGL(
                                (lattice_point_major<BK.value, SH.value, SX.value, WU.value, WF.value, V16.value>),
                                dim3(gx), dim3(kWave * kPmWaves), 0, hs, generator, s, first32, nn, shifts, out_u32,
                                out_f32, ld);
                        });
                    } else if (fast) {
                        with_bool(ctx->lattice_tune.nontemporal != 0, [&](auto NT) {
                            uint32_t nchunks;
                            const GenTune tn = launch_tune(ctx->lattice_tune, WU.value && WF.value);
                            const dim3 grid = fast_grid(nn, s, tn, &nchunks);
                            hipLaunchKernelGGL(
                                (lattice_fast<BK.value, SH.value, SX.value, WU.value, WF.value, NT.value>), grid,
                                dim3(kWave), 0, hs, generator, first32, nn, shifts, out_u32, out_f32, ld,
                                tn.chunks_per_wave, nchunks);
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

namespace qmc {
namespace {

// Shared argument checks of the partitioned calls; sets *r = rev_q(part).
qmc_status validate_partition(const char* who, uint32_t index_bits, uint32_t q, uint32_t part, uint32_t* r) {
    if (q > 32 || q > index_bits)
        return fail(QMC_ERR_OUT_OF_RANGE, "%s: log2_parts = %u outside [0, min(32, %u)]", who, q, index_bits);
    if (q < 32 && part >> q)
        return fail(QMC_ERR_OUT_OF_RANGE, "%s: part %u outside [0, 2^%u)", who, part, q);
    uint32_t v = 0;
    for (uint32_t k = 0; k < q; ++k) v |= ((part >> k) & 1u) << (q - 1 - k);
    *r = v;
    return QMC_OK;
}

// Runs launch(first, count, offset) over pieces of at most 2^31 points.
template <typename F>
void over_pieces(uint64_t first, uint64_t n, F&& launch) {
    const uint64_t piece = uint64_t(1) << 31;
    for (uint64_t done = 0; done < n; done += piece)
        launch(first + done, static_cast<uint32_t>(std::min(piece, n - done)), done);
}

}  // namespace
}  // namespace qmc

extern "C" qmc_status qmc_generate_sobol64(qmc_context ctx, qmc_stream stream, const uint32_t* matrices,
                                           uint32_t columns, uint32_t s, uint32_t log2_parts, uint32_t part,
                                           uint64_t first, uint64_t n, const uint32_t* nus_seeds,
                                           const uint32_t* shifts, uint32_t flags, uint32_t* out_u32,
                                           float* out_f32, uint64_t ld) {
    const char* who = "qmc_generate_sobol64";
    if (columns == 0 || columns > 64)
        return fail(QMC_ERR_OUT_OF_RANGE, "%s: columns = %u outside [1, 64]", who, columns);
    uint32_t r = 0;
    qmc_status st = validate_partition(who, columns, log2_parts, part, &r);
    if (st != QMC_OK) return st;
    st = validate_generation(who, ctx, matrices, uint64_t(columns) * 4, s, first, n, flags, QMC_SHIFT_XOR, nus_seeds,
                             shifts, out_u32, out_f32, ld, columns - log2_parts);
    if (st != QMC_OK || n == 0) return st;
    DeviceGuard guard(ctx->device);
    if (guard.status != QMC_OK) return guard.status;
    hipStream_t hs = as_stream(stream);
    const bool nus = nus_seeds != nullptr, shift = shifts != nullptr, sxor = (flags & QMC_SHIFT_XOR) != 0;
    const bool fast = (first % 4 == 0) && (ld % 4 == 0) && aligned16(out_u32) && aligned16(out_f32);
    const uint32_t q = log2_parts;
    clear_launch_error();
    with_bool(nus, [&](auto NUS) {
        with_bool(shift, [&](auto SH) {
            with_bool(sxor && shift, [&](auto SX) {
                with_outputs(out_u32 != nullptr, out_f32 != nullptr, [&](auto WU, auto WF) {
                    over_pieces(first, n, [&](uint64_t f, uint32_t nn, uint64_t off) {
                        uint32_t* ou = out_u32 ? out_u32 + off : nullptr;
                        float* of = out_f32 ? out_f32 + off : nullptr;
                        if (fast) {
                            with_bool(ctx->sobol_tune.nontemporal != 0, [&](auto NT) {
                                uint32_t nchunks;
                                const GenTune tn = launch_tune(ctx->sobol_tune, WU.value && WF.value);
                                const dim3 grid = fast_grid(nn, s, tn, &nchunks);
                                hipLaunchKernelGGL(
                                    (sobol64_fast<NUS.value, SH.value, SX.value, WU.value, WF.value, NT.value>), grid,
                                    dim3(kWave), 0, hs, matrices, columns, q, r, f, nn, nus_seeds, shifts, ou, of, ld,
                                    tn.chunks_per_wave, nchunks);
                            });
                        } else {
                            hipLaunchKernelGGL((sobol64_general<NUS.value, SH.value, SX.value, WU.value, WF.value>),
                                               dim3(general_grid(ctx, nn)), dim3(kBlock), 0, hs, matrices, columns, s,
                                               q, r, f, nn, nus_seeds, shifts, ou, of, ld);
                        }
                    });
                });
            });
        });
    });
    return check_launch(who);
}

extern "C" qmc_status qmc_generate_lattice64(qmc_context ctx, qmc_stream stream, const uint32_t* generator,
                                             uint32_t s, uint32_t log2_parts, uint32_t part, uint64_t first,
                                             uint64_t n, const uint32_t* shifts, uint32_t flags, uint32_t* out_u32,
                                             float* out_f32, uint64_t ld) {
    const char* who = "qmc_generate_lattice64";
    uint32_t r = 0;
    qmc_status st = validate_partition(who, 64, log2_parts, part, &r);
    if (st != QMC_OK) return st;
    st = validate_generation(who, ctx, generator, 4, s, first, n, flags, QMC_SHIFT_XOR | QMC_LATTICE_BACKWARD, shifts,
                             nullptr, out_u32, out_f32, ld, 64 - log2_parts);
    if (st != QMC_OK || n == 0) return st;
    DeviceGuard guard(ctx->device);
    if (guard.status != QMC_OK) return guard.status;
    hipStream_t hs = as_stream(stream);
    const bool back = (flags & QMC_LATTICE_BACKWARD) != 0, shift = shifts != nullptr;
    const bool sxor = (flags & QMC_SHIFT_XOR) != 0;
    const bool fast = (first % 4 == 0) && (ld % 4 == 0) && aligned16(out_u32) && aligned16(out_f32);
    const uint32_t q = log2_parts;
    clear_launch_error();
    with_bool(back, [&](auto BK) {
        with_bool(shift, [&](auto SH) {
            with_bool(sxor && shift, [&](auto SX) {
                with_outputs(out_u32 != nullptr, out_f32 != nullptr, [&](auto WU, auto WF) {
                    over_pieces(first, n, [&](uint64_t f, uint32_t nn, uint64_t off) {
                        uint32_t* ou = out_u32 ? out_u32 + off : nullptr;
                        float* of = out_f32 ? out_f32 + off : nullptr;
                        if (fast) {
                            with_bool(ctx->lattice_tune.nontemporal != 0, [&](auto NT) {
                                uint32_t nchunks;
                                const GenTune tn = launch_tune(ctx->lattice_tune, WU.value && WF.value);
                                const dim3 grid = fast_grid(nn, s, tn, &nchunks);
                                hipLaunchKernelGGL(
                                    (lattice64_fast<BK.value, SH.value, SX.value, WU.value, WF.value, NT.value>), grid,
                                    dim3(kWave), 0, hs, generator, q, r, f, nn, shifts, ou, of, ld,
                                    tn.chunks_per_wave, nchunks);
                            });
                        } else {
                            hipLaunchKernelGGL((lattice64_general<BK.value, SH.value, SX.value, WU.value, WF.value>),
                                               dim3(general_grid(ctx, nn)), dim3(kBlock), 0, hs, generator, s, q, r,
                                               f, nn, shifts, ou, of, ld);
                        }
                    });
                });
            });
        });
    });
    return check_launch(who);
}

extern "C" qmc_status qmc_generate_halton(qmc_context ctx, qmc_stream stream, uint32_t s, uint64_t first, uint64_t n,
                                          uint32_t mode, const uint32_t* factors, uint32_t* out_u32, float* out_f32,
                                          uint64_t ld) {
    const char* who = "qmc_generate_halton";
    if (mode > QMC_HALTON_LINEAR) return fail(QMC_ERR_INVALID_ARGUMENT, "%s: unknown permutation mode %u", who, mode);
    if (mode == QMC_HALTON_LINEAR && !factors && n)
        return fail(QMC_ERR_INVALID_ARGUMENT, "%s: linear scrambling needs factors", who);
    // validate_generation wants a table; the factors (or any non-NULL marker) stand in for it
    static const uint32_t marker = 0;
    qmc_status st = validate_generation(who, ctx, factors ? static_cast<const void*>(factors) : &marker,
                                        factors ? 4 : 0, s, first, n, 0, 0, nullptr, nullptr, out_u32, out_f32, ld);
    if (st != QMC_OK || n == 0) return st;
    if (n > (uint64_t(1) << 31)) {
        const uint64_t hh = uint64_t(1) << 31;
        st = qmc_generate_halton(ctx, stream, s, first, hh, mode, factors, out_u32, out_f32, ld);
        if (st != QMC_OK) return st;
        return qmc_generate_halton(ctx, stream, s, first + hh, n - hh, mode, factors,
                                   out_u32 ? out_u32 + hh : nullptr, out_f32 ? out_f32 + hh : nullptr, ld);
    }
    DeviceGuard guard(ctx->device);
    if (guard.status != QMC_OK) return guard.status;
    hipStream_t hs = as_stream(stream);
    const bool fast = (first % 4 == 0) && (ld % 4 == 0) && aligned16(out_u32) && aligned16(out_f32);
    const uint32_t first32 = static_cast<uint32_t>(first);
    const uint32_t nn = static_cast<uint32_t>(n);
    // linear digit permutations are formed per wavefront: longer runs amortise them
    const uint32_t run = mode == QMC_HALTON_LINEAR ? 8u : 4u;
    HaltonTable tab{};
    if (fast) halton_table(s, run, &tab);
    clear_launch_error();
    auto launch = [&](auto MODE) {
        with_outputs(out_u32 != nullptr, out_f32 != nullptr, [&](auto WU, auto WF) {
            if (fast) {
                const uint32_t nchunks = static_cast<uint32_t>((n + kChunk - 1) / kChunk);
                hipLaunchKernelGGL((halton_fast<decltype(MODE)::value, WU.value, WF.value, false>),
                                   dim3((nchunks + run - 1) / run, s), dim3(kWave), 0, hs, first32, nn, factors,
                                   out_u32, out_f32, ld, run, nchunks, tab);
            } else {
                const uint64_t want = (n + kWave - 1) / kWave;
                const uint32_t gx = static_cast<uint32_t>(std::min<uint64_t>(want, uint64_t(ctx->num_cus) * 16));
                hipLaunchKernelGGL((halton_general<decltype(MODE)::value, WU.value, WF.value>), dim3(gx, s),
                                   dim3(kWave), 0, hs, first32, nn, factors, out_u32, out_f32, ld);
            }
        });
    };
    if (mode == QMC_HALTON_FAURE)
        launch(std::integral_constant<uint32_t, 1>{});
    else if (mode == QMC_HALTON_LINEAR)
        launch(std::integral_constant<uint32_t, 2>{});
    else
        launch(std::integral_constant<uint32_t, 0>{});
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
