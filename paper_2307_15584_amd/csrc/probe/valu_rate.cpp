// Issue rate of single VALU instructions on this GPU: the ceiling against which the per-pixel
// kernels' VALU roofline is priced.  Every lane runs eight independent chains of one instruction
// (so dependences do not limit issue).  One block per compute unit (its LDS request leaves room
// for no second block), with the same number of wavefronts on each SIMD, and loops long enough
// (a few milliseconds per launch) that launch and ramp-up do not matter.  Prints wave64
// instructions per compute unit per nanosecond of wall time; divided by the shader clock
// (GRBM_GUI_ACTIVE / 8 dies / duration under rocprofv3 --pmc) it is the rate per cycle.
//
//   valu_rate [waves_per_simd]     prints a markdown table
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <vector>

#define CHECK(x)                                                                              \
    do {                                                                                      \
        hipError_t e_ = (x);                                                                  \
        if (e_ != hipSuccess) {                                                               \
            std::fprintf(stderr, "%s:%d: %s: %s\n", __FILE__, __LINE__, #x, hipGetErrorString(e_)); \
            std::exit(1);                                                                     \
        }                                                                                     \
    } while (0)

constexpr int kIters = 8192;  // loop trips
constexpr int kUnroll = 8;    // instructions per chain per trip
constexpr int kChains = 8;    // independent chains per lane
constexpr int kPerWave = kIters * kUnroll * kChains;

// One instruction of the kind under test on chain register r; a, b: loop-invariant sources.
#define OP(name, text)                                                                         \
    struct name {                                                                             \
        static constexpr const char* label = text;                                            \
        __device__ static void run(uint32_t& r, uint32_t a, uint32_t b);                      \
    };
OP(AddU32, "v_add_u32")
OP(AddF32, "v_add_f32")
OP(MulF32, "v_mul_f32")
OP(XorB32, "v_xor_b32")
OP(FmaF32, "v_fma_f32")
OP(FmacF32, "v_fmac_f32")
OP(MadU24, "v_mad_u32_u24")
OP(MulLoU32, "v_mul_lo_u32")
OP(LshlB32, "v_lshlrev_b32")
OP(BfrevB32, "v_bfrev_b32")
OP(FfbhU32, "v_ffbh_u32")
OP(CvtF32U32, "v_cvt_f32_u32")
OP(ExpF32, "v_exp_f32")
OP(CosF32, "v_cos_f32")
#undef OP

__device__ void AddU32::run(uint32_t& r, uint32_t a, uint32_t) { asm volatile("v_add_u32 %0, %0, %1" : "+v"(r) : "v"(a)); }
__device__ void AddF32::run(uint32_t& r, uint32_t a, uint32_t) { asm volatile("v_add_f32 %0, %0, %1" : "+v"(r) : "v"(a)); }
__device__ void MulF32::run(uint32_t& r, uint32_t a, uint32_t) { asm volatile("v_mul_f32 %0, %0, %1" : "+v"(r) : "v"(a)); }
__device__ void XorB32::run(uint32_t& r, uint32_t a, uint32_t) { asm volatile("v_xor_b32 %0, %0, %1" : "+v"(r) : "v"(a)); }
__device__ void FmaF32::run(uint32_t& r, uint32_t a, uint32_t b) { asm volatile("v_fma_f32 %0, %0, %1, %2" : "+v"(r) : "v"(a), "v"(b)); }
__device__ void FmacF32::run(uint32_t& r, uint32_t a, uint32_t b) { asm volatile("v_fmac_f32 %0, %1, %2" : "+v"(r) : "v"(a), "v"(b)); }
__device__ void MadU24::run(uint32_t& r, uint32_t a, uint32_t b) { asm volatile("v_mad_u32_u24 %0, %0, %1, %2" : "+v"(r) : "v"(a), "v"(b)); }
__device__ void MulLoU32::run(uint32_t& r, uint32_t a, uint32_t) { asm volatile("v_mul_lo_u32 %0, %0, %1" : "+v"(r) : "v"(a)); }
__device__ void LshlB32::run(uint32_t& r, uint32_t a, uint32_t) { asm volatile("v_lshlrev_b32 %0, %1, %0" : "+v"(r) : "v"(a)); }
__device__ void BfrevB32::run(uint32_t& r, uint32_t, uint32_t) { asm volatile("v_bfrev_b32 %0, %0" : "+v"(r)); }
__device__ void FfbhU32::run(uint32_t& r, uint32_t, uint32_t) { asm volatile("v_ffbh_u32 %0, %0" : "+v"(r)); }
__device__ void CvtF32U32::run(uint32_t& r, uint32_t, uint32_t) { asm volatile("v_cvt_f32_u32 %0, %0" : "+v"(r)); }
__device__ void ExpF32::run(uint32_t& r, uint32_t, uint32_t) { asm volatile("v_exp_f32 %0, %0" : "+v"(r)); }
__device__ void CosF32::run(uint32_t& r, uint32_t, uint32_t) { asm volatile("v_cos_f32 %0, %0" : "+v"(r)); }

// sink keeps the chains live.
template <typename Op>
__global__ __launch_bounds__(1024) void issue(uint32_t* sink, uint32_t seed) {
    uint32_t r[kChains];
    const uint32_t a = seed | 1u, b = seed >> 3;
#pragma unroll
    for (int c = 0; c < kChains; ++c) r[c] = threadIdx.x * 2654435761u + c;
    __syncthreads();
    for (int it = 0; it < kIters; ++it) {
#pragma unroll
        for (int u = 0; u < kUnroll; ++u)
#pragma unroll
            for (int c = 0; c < kChains; ++c) Op::run(r[c], a, b);
    }
    uint32_t x = 0;
#pragma unroll
    for (int c = 0; c < kChains; ++c) x ^= r[c];
    if (x == 0x12345678u) sink[0] = x;
}

// The inner step of the lobe integrand: t = y s + b, e += t t for 32 dimensions, with y, s and
// b in 96 distinct registers (each FMA reads three registers) and C exponent chains taking the
// dimensions in turn, so that consecutive updates of one chain are 2C instructions apart.
// 64 instructions per step.
constexpr int kLobeDims = 32;
constexpr int kLobeIters = kIters * kUnroll * kChains / (2 * kLobeDims);

template <int C>
__device__ __forceinline__ void lobe_group(float (&e)[C], const float* y, const float* s, const float* b);
template <>
__device__ __forceinline__ void lobe_group<1>(float (&e)[1], const float* y, const float* s, const float* b) {
    float t0;
    asm volatile("v_fma_f32 %0, %2, %3, %4\n\tv_fmac_f32 %1, %0, %0" : "=&v"(t0), "+v"(e[0]) : "v"(y[0]), "v"(s[0]), "v"(b[0]));
}
template <>
__device__ __forceinline__ void lobe_group<2>(float (&e)[2], const float* y, const float* s, const float* b) {
    float t0, t1;
    asm volatile(
        "v_fma_f32 %0, %4, %5, %6\n\tv_fma_f32 %1, %7, %8, %9\n\t"
        "v_fmac_f32 %2, %0, %0\n\tv_fmac_f32 %3, %1, %1"
        : "=&v"(t0), "=&v"(t1), "+v"(e[0]), "+v"(e[1])
        : "v"(y[0]), "v"(s[0]), "v"(b[0]), "v"(y[1]), "v"(s[1]), "v"(b[1]));
}
template <>
__device__ __forceinline__ void lobe_group<4>(float (&e)[4], const float* y, const float* s, const float* b) {
    float e01[2] = {e[0], e[1]}, e23[2] = {e[2], e[3]};
    float t0, t1, t2, t3;
    asm volatile(
        "v_fma_f32 %0, %8, %9, %10\n\tv_fma_f32 %1, %11, %12, %13\n\t"
        "v_fma_f32 %2, %14, %15, %16\n\tv_fma_f32 %3, %17, %18, %19\n\t"
        "v_fmac_f32 %4, %0, %0\n\tv_fmac_f32 %5, %1, %1\n\t"
        "v_fmac_f32 %6, %2, %2\n\tv_fmac_f32 %7, %3, %3"
        : "=&v"(t0), "=&v"(t1), "=&v"(t2), "=&v"(t3), "+v"(e01[0]), "+v"(e01[1]), "+v"(e23[0]), "+v"(e23[1])
        : "v"(y[0]), "v"(s[0]), "v"(b[0]), "v"(y[1]), "v"(s[1]), "v"(b[1]),
          "v"(y[2]), "v"(s[2]), "v"(b[2]), "v"(y[3]), "v"(s[3]), "v"(b[3]));
    e[0] = e01[0];
    e[1] = e01[1];
    e[2] = e23[0];
    e[3] = e23[1];
}

template <int C>
__global__ __launch_bounds__(1024) void issue_lobe(uint32_t* sink, uint32_t seed) {
    float y[kLobeDims], s[kLobeDims], b[kLobeDims];
#pragma unroll
    for (int j = 0; j < kLobeDims; ++j) {
        y[j] = float(threadIdx.x + j) * 0x1p-10f;
        s[j] = float(seed + j) * 0x1p-12f;
        b[j] = -float(seed ^ j) * 0x1p-14f;
    }
    float e[C];
#pragma unroll
    for (int c = 0; c < C; ++c) e[c] = 0.0f;
    __syncthreads();
    for (int it = 0; it < kLobeIters; ++it) {
#pragma unroll
        for (int j = 0; j < kLobeDims; j += C) lobe_group<C>(e, y + j, s + j, b + j);
    }
    float x = 0.0f;
#pragma unroll
    for (int c = 0; c < C; ++c) x += e[c];
    if (x == 1.2345f) sink[0] = 1u;
}

template <int C>
struct LobeStep {
    static constexpr int chains = C;
    static constexpr const char* label = C == 1 ? "lobe step, 1 exponent chain (`v_fma_f32 t, y, s, b` + `v_fmac_f32 e, t, t`)"
                                       : C == 2 ? "lobe step, 2 exponent chains" : "lobe step, 4 exponent chains";
};
template <typename T>
struct IsLobe : std::false_type {};
template <int C>
struct IsLobe<LobeStep<C>> : std::true_type {};

template <typename Op>
void measure(int cus, int waves_per_simd, size_t lds, uint32_t* d_sink) {
    const int blocks = cus;                  // one block per compute unit
    const int threads = 256 * waves_per_simd;  // waves_per_simd wavefronts on each of the 4 SIMDs
    auto launch = [&](uint32_t seed) {
        if constexpr (IsLobe<Op>::value)
            hipLaunchKernelGGL(issue_lobe<Op::chains>, dim3(blocks), dim3(threads), lds, 0, d_sink, seed);
        else
            hipLaunchKernelGGL(issue<Op>, dim3(blocks), dim3(threads), lds, 0, d_sink, seed);
    };
    launch(12345u);  // warm-up
    CHECK(hipDeviceSynchronize());
    hipEvent_t e0, e1;
    CHECK(hipEventCreate(&e0));
    CHECK(hipEventCreate(&e1));
    CHECK(hipEventRecord(e0));
    launch(777u);
    CHECK(hipEventRecord(e1));
    CHECK(hipEventSynchronize(e1));
    CHECK(hipGetLastError());
    float ms = 0;
    CHECK(hipEventElapsedTime(&ms, e0, e1));
    CHECK(hipEventDestroy(e0));
    CHECK(hipEventDestroy(e1));
    // every CU runs 4 * waves_per_simd wavefronts, each issuing kPerWave instructions
    const double per_cu_ns = 4.0 * waves_per_simd * kPerWave / (ms * 1e6);
    std::printf("| `%s` | %.3f | %.3f |\n", Op::label, per_cu_ns, ms);
}

int main(int argc, char** argv) {
    const int wps = std::min(4, std::max(1, argc > 1 ? std::atoi(argv[1]) : 4));
    hipDeviceProp_t prop;
    CHECK(hipGetDeviceProperties(&prop, 0));
    const int cus = prop.multiProcessorCount;
    const size_t lds = prop.maxSharedMemoryPerMultiProcessor / 2 + 1024;
    if (lds > prop.sharedMemPerBlock) {
        std::fprintf(stderr, "cannot request %zu bytes of LDS per block (at most %zu)\n", lds, prop.sharedMemPerBlock);
        return 1;
    }
    uint32_t* d_sink = nullptr;
    CHECK(hipMalloc(&d_sink, 64));
    std::printf("%s, %d compute units, %d wavefronts per SIMD, %d instructions per wavefront, %zu B of LDS per "
                "block\n\n", prop.gcnArchName, cus, wps, kPerWave, lds);
    std::printf("| Instruction | wave64 instr / CU / ns | kernel ms |\n");
    std::printf("|---|---:|---:|\n");
    measure<AddU32>(cus, wps, lds, d_sink);
    measure<AddF32>(cus, wps, lds, d_sink);
    measure<MulF32>(cus, wps, lds, d_sink);
    measure<XorB32>(cus, wps, lds, d_sink);
    measure<FmaF32>(cus, wps, lds, d_sink);
    measure<FmacF32>(cus, wps, lds, d_sink);
    measure<MadU24>(cus, wps, lds, d_sink);
    measure<MulLoU32>(cus, wps, lds, d_sink);
    measure<LshlB32>(cus, wps, lds, d_sink);
    measure<BfrevB32>(cus, wps, lds, d_sink);
    measure<FfbhU32>(cus, wps, lds, d_sink);
    measure<CvtF32U32>(cus, wps, lds, d_sink);
    measure<ExpF32>(cus, wps, lds, d_sink);
    measure<CosF32>(cus, wps, lds, d_sink);
    measure<LobeStep<1>>(cus, wps, lds, d_sink);
    measure<LobeStep<2>>(cus, wps, lds, d_sink);
    measure<LobeStep<4>>(cus, wps, lds, d_sink);
    CHECK(hipFree(d_sink));
    return 0;
}
