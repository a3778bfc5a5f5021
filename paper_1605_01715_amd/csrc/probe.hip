// Issue-rate probes: a measurement utility, not a step of the method.
//
// Every lane runs independent float32 (or 32-bit integer) chains, so the
// only limit is how fast a SIMD issues the instructions; one more kind runs
// bfloat16 matrix products on operands held in registers. The rates they
// reach are the ceilings against which the leaf evaluation (a loop of
// float32 VALU instructions with one reciprocal square root per pair) is
// judged: packed float32 is not used anywhere in the library, so the
// chip's float32 peak, which counts it, is not reachable by that loop.
#include "probe.hpp"

namespace fmm {

namespace {

// 16 chains of v_fma_f32
__global__ __launch_bounds__(256) void k_probe_fma(float *out, float a, float b, int iters) {
    float acc[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[i] = threadIdx.x * 1e-3f + i;
    for (int it = 0; it < iters; ++it)
#pragma unroll
        for (int i = 0; i < 16; ++i) acc[i] = __builtin_fmaf(acc[i], a, b);
    float s = 0.f;
#pragma unroll
    for (int i = 0; i < 16; ++i) s += acc[i];
    out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// 16 chains of v_rsq_f32
__global__ __launch_bounds__(256) void k_probe_rsq(float *out, float a, float b, int iters) {
    float acc[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[i] = threadIdx.x * 1e-3f + i + 1.f;
    for (int it = 0; it < iters; ++it)
#pragma unroll
        for (int i = 0; i < 16; ++i) acc[i] = __builtin_amdgcn_rsqf(acc[i]);
    float s = a + b;
#pragma unroll
    for (int i = 0; i < 16; ++i) s += acc[i];
    out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// 8 chains, each step 12 v_fma_f32 then one v_rsq_f32 (the pair loop's ratio)
__global__ __launch_bounds__(256) void k_probe_mix(float *out, float a, float b, int iters) {
    float acc[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) acc[i] = threadIdx.x * 1e-3f + i + 1.f;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int r = 0; r < 12; ++r)
#pragma unroll
            for (int i = 0; i < 8; ++i) acc[i] = __builtin_fmaf(acc[i], a, b);
#pragma unroll
        for (int i = 0; i < 8; ++i) acc[i] = __builtin_amdgcn_rsqf(acc[i]);
    }
    float s = 0.f;
#pragma unroll
    for (int i = 0; i < 8; ++i) s += acc[i];
    out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// 8 chains, each step a 32-bit add then an exclusive or
__global__ __launch_bounds__(256) void k_probe_int(float *out, uint32_t a, uint32_t b, int iters) {
    uint32_t acc[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) acc[i] = threadIdx.x * 2654435761u + i;
    for (int it = 0; it < iters; ++it)
#pragma unroll
        for (int i = 0; i < 8; ++i) acc[i] = (acc[i] + a) ^ b;
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < 8; ++i) s ^= acc[i];
    out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = (float)s;
}

typedef __bf16 pbf16x8 __attribute__((ext_vector_type(8)));
typedef float pf32x16 __attribute__((ext_vector_type(16)));

// 4 independent accumulators of v_mfma_f32_32x32x16_bf16, operands held in
// registers: the matrix-core rate with no data movement at all
__global__ __launch_bounds__(256) void k_probe_mfma(float *out, float a, float b, int iters) {
    pbf16x8 va, vb;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        va[k] = (__bf16)a;
        vb[k] = (__bf16)b;
    }
    pf32x16 acc[4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[i][v] = 0.f;
    for (int it = 0; it < iters; ++it)
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[i] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(va, vb, acc[i], 0, 0, 0);
    float s = 0.f;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int v = 0; v < 16; ++v) s += acc[i][v];
    out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

}  // namespace

int64_t issue_probe_instr(int kind) { return kind == 2 ? 104 : kind == 4 ? 4 : 16; }

void issue_probe(int kind, int64_t nthreads, int iters, float *out, hipStream_t s) {
    const dim3 grid((unsigned)(nthreads / 256)), block(256);
    switch (kind) {
    case 0: hipLaunchKernelGGL(k_probe_fma, grid, block, 0, s, out, 0.999f, 1e-3f, iters); break;
    case 1: hipLaunchKernelGGL(k_probe_rsq, grid, block, 0, s, out, 0.999f, 1e-3f, iters); break;
    case 2: hipLaunchKernelGGL(k_probe_mix, grid, block, 0, s, out, 0.999f, 1e-3f, iters); break;
    case 3: hipLaunchKernelGGL(k_probe_int, grid, block, 0, s, out, 0x9e3779b9u, 0x85ebca6bu, iters); break;
    default: hipLaunchKernelGGL(k_probe_mfma, grid, block, 0, s, out, 1.0f, 0.5f, iters); break;
    }
    FMM_HIP(hipGetLastError());
}

}  // namespace fmm
