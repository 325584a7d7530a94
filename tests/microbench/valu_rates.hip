// valu_rates.hip -- issue rates of the integer VALU instructions the block
// update is built from, on the GPU it runs on.  Each kernel runs eight
// independent dependency chains per thread over a grid of many waves per
// SIMD, so latency is hidden and the time measures throughput.  Rates are
// wave64 instructions x 64 lanes per second (all instructions of a step
// counted, as listed); the ratio column is the rate over that of v_xad_u32
// (a full-rate 32-bit instruction): 1.0 means every instruction of the step
// issues at full rate, 0.67 for a two-instruction step would mean one of
// them takes two issue slots.
//
// A measurement helper, not part of the library (nothing builds or loads it
// automatically).  Build and run from the repository root:
//   hipcc --offload-arch=gfx950 -O3 -Xclang -target-feature -Xclang
//     -packed-fp32-ops tests/microbench/valu_rates.hip -o /tmp/valu_rates
//   /tmp/valu_rates
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>

#define CHECK(x)                                                              \
    do {                                                                      \
        hipError_t e_ = (x);                                                  \
        if (e_ != hipSuccess) {                                               \
            std::printf("HIP error %s at line %d\n", hipGetErrorString(e_),   \
                        __LINE__);                                            \
            return 1;                                                         \
        }                                                                     \
    } while (0)

namespace {

constexpr int kChains = 8;

// v_xad_u32: (a ^ m) + j, one instruction per chain step
__global__ void k_xad(uint32_t *out, int iters, uint32_t m)
{
    uint32_t a[kChains];
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
#pragma unroll
    for (int j = 0; j < kChains; ++j)
        a[j] = tid + j;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int j = 0; j < kChains; ++j)
            a[j] = (a[j] ^ m) + (uint32_t)j;
    }
    uint32_t r = 0;
#pragma unroll
    for (int j = 0; j < kChains; ++j)
        r ^= a[j];
    out[tid] = r;
}

// v_mad_u64_u32: 32 x 32 -> 64-bit product, then the two halves xored
// (v_xor_b32): two instructions per step, as in a Philox round
__global__ void k_mad64(uint32_t *out, int iters, uint32_t m)
{
    uint32_t a[kChains];
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
#pragma unroll
    for (int j = 0; j < kChains; ++j)
        a[j] = tid + j;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int j = 0; j < kChains; ++j) {
            const uint64_t p = (uint64_t)m * a[j];
            a[j] = (uint32_t)(p >> 32) ^ (uint32_t)p;
        }
    }
    uint32_t r = 0;
#pragma unroll
    for (int j = 0; j < kChains; ++j)
        r ^= a[j];
    out[tid] = r;
}

// v_mul_hi_u32 (with a v_add_u32 to keep the chain going: two instructions)
__global__ void k_mulhi(uint32_t *out, int iters, uint32_t m)
{
    uint32_t a[kChains];
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
#pragma unroll
    for (int j = 0; j < kChains; ++j)
        a[j] = tid + j;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int j = 0; j < kChains; ++j)
            a[j] = __umulhi(a[j], m) + a[j];
    }
    uint32_t r = 0;
#pragma unroll
    for (int j = 0; j < kChains; ++j)
        r ^= a[j];
    out[tid] = r;
}

// v_perm_b32 with a per-chain selector
__global__ void k_perm(uint32_t *out, int iters, uint32_t m)
{
    uint32_t a[kChains];
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
#pragma unroll
    for (int j = 0; j < kChains; ++j)
        a[j] = tid + j;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int j = 0; j < kChains; ++j)
            a[j] = __builtin_amdgcn_perm(a[j], m, 0x05040100u + (uint32_t)j);
    }
    uint32_t r = 0;
#pragma unroll
    for (int j = 0; j < kChains; ++j)
        r ^= a[j];
    out[tid] = r;
}

// v_dot4_u32_u8 accumulating into the chain
__global__ void k_dot4(uint32_t *out, int iters, uint32_t m)
{
    uint32_t a[kChains];
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
#pragma unroll
    for (int j = 0; j < kChains; ++j)
        a[j] = tid + j;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int j = 0; j < kChains; ++j)
            a[j] = __builtin_amdgcn_udot4(a[j], m, a[j], false);
    }
    uint32_t r = 0;
#pragma unroll
    for (int j = 0; j < kChains; ++j)
        r ^= a[j];
    out[tid] = r;
}

} // namespace

int main()
{
    int dev = 0;
    hipDeviceProp_t prop;
    CHECK(hipGetDevice(&dev));
    CHECK(hipGetDeviceProperties(&prop, dev));
    const int cus = prop.multiProcessorCount;
    const int threads = 256, blocks = cus * 16; // 16 waves per SIMD
    const int iters = 4000;
    uint32_t *out = nullptr;
    CHECK(hipMalloc(&out, (size_t)blocks * threads * 4));
    hipEvent_t e0, e1;
    CHECK(hipEventCreate(&e0));
    CHECK(hipEventCreate(&e1));
    std::printf("device %s, %d CUs, %d x %d threads, %d iterations, %d "
                "chains per thread\n",
                prop.gcnArchName, cus, blocks, threads, iters, kChains);
    std::printf("%-24s %10s %14s %8s\n", "instruction", "ms",
                "lane-instr/s", "ratio");
    double ref = 0;
    auto time_one = [&](const char *name, auto kern,
                        double instr_per_chain_step) -> int {
        hipLaunchKernelGGL(kern, dim3(blocks), dim3(threads), 0, 0, out,
                           iters / 10, 0xD2511F53u);
        CHECK(hipGetLastError());
        CHECK(hipDeviceSynchronize());
        CHECK(hipEventRecord(e0));
        hipLaunchKernelGGL(kern, dim3(blocks), dim3(threads), 0, 0, out,
                           iters, 0xD2511F53u);
        CHECK(hipGetLastError());
        CHECK(hipEventRecord(e1));
        CHECK(hipEventSynchronize(e1));
        float ms = 0;
        CHECK(hipEventElapsedTime(&ms, e0, e1));
        const double lanes = (double)blocks * threads * iters * kChains *
                             instr_per_chain_step;
        const double rate = lanes / (ms * 1e-3);
        if (ref == 0)
            ref = rate;
        std::printf("%-24s %10.3f %14.4e %8.3f\n", name, ms, rate,
                    rate / ref);
        return 0;
    };
    if (time_one("v_xad_u32", k_xad, 1.0) ||
        time_one("v_mad_u64_u32 + v_xor", k_mad64, 2.0) ||
        time_one("v_mul_hi_u32 + v_add", k_mulhi, 2.0) ||
        time_one("v_perm_b32", k_perm, 1.0) ||
        time_one("v_dot4_u32_u8", k_dot4, 1.0))
        return 1;
    CHECK(hipFree(out));
    return 0;
}
