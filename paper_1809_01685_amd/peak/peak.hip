// Achievable arithmetic peaks of one MI355X, for the roofline's second
// denominator: every wave runs NCH independent accumulator chains of one
// instruction for `iters` rounds, so the issue rate, not the dependency
// latency, bounds the loop.  The operands come from the thread index and a
// runtime scale (nothing folds at compile time), and every accumulator is
// summed into out[] at the end so that no chain is dead.
//
// kind 0: v_mfma_f32_16x16x32_bf16   16384 flops per instruction per wave
// kind 1: v_mfma_f32_16x16x4_f32      2048
// kind 2: v_mfma_f64_16x16x4_f64      2048
// kind 3: v_fma_f64 (vector ALU)      2 per lane, 128 per wave
// kind 4: v_fma_f32 (vector ALU)      2 per lane, 128 per wave (packed forms
//         are disabled in this library's compile flags, so this is the unpacked rate)
// kind 5: v_mfma_f32_32x32x16_bf16   32768 (four accumulator chains of 16)
//
// Built with the matrix instructions' VGPR form (-amdgpu-mfma-vgpr-form): in
// the accumulator-register form the loop-carried accumulators were copied
// between register files every round, which the contraction kernels (VGPR
// form already) do not do.
//
// Exported as plain C: tnslq_peak_flops_per_round(kind) gives the flops one
// wave does per round; tnslq_peak_launch(kind, blocks, iters, scale, out,
// stream) launches `blocks` workgroups of 256 threads (4 waves) and writes
// one float per thread into out (blocks * 256 entries, device).
#include <hip/hip_runtime.h>
#include <stdint.h>

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(4))) float f32x4;
typedef __attribute__((ext_vector_type(4))) double f64x4;
typedef __attribute__((ext_vector_type(16))) float f32x16;

namespace {

constexpr int NCH = 8;

__global__ void __launch_bounds__(256) k_peak_bf16(int iters, float scale, float *out) {
    const float v = scale * (float)(threadIdx.x + 1);
    bf16x8 a, b;
    for (int i = 0; i < 8; ++i) {
        a[i] = (__bf16)(v * (float)(i + 1));
        b[i] = (__bf16)(v * (float)(8 - i));
    }
    f32x4 acc[NCH];
#pragma unroll
    for (int c = 0; c < NCH; ++c) acc[c] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int c = 0; c < NCH; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[c], 0, 0, 0);
    }
    float s = 0.f;
#pragma unroll
    for (int c = 0; c < NCH; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
    out[(size_t)blockIdx.x * 256 + threadIdx.x] = s;
}

__global__ void __launch_bounds__(256) k_peak_bf16_32(int iters, float scale, float *out) {
    const float v = scale * (float)(threadIdx.x + 1);
    bf16x8 a, b;
    for (int i = 0; i < 8; ++i) {
        a[i] = (__bf16)(v * (float)(i + 1));
        b[i] = (__bf16)(v * (float)(8 - i));
    }
    f32x16 acc[4];
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int e = 0; e < 16; ++e) acc[c][e] = 0.f;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc[c], 0, 0, 0);
    }
    float s = 0.f;
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int e = 0; e < 16; ++e) s += acc[c][e];
    out[(size_t)blockIdx.x * 256 + threadIdx.x] = s;
}

__global__ void __launch_bounds__(256) k_peak_f32(int iters, float scale, float *out) {
    const float a = scale * (float)(threadIdx.x + 1), b = scale * (float)(threadIdx.x + 2);
    f32x4 acc[NCH];
#pragma unroll
    for (int c = 0; c < NCH; ++c) acc[c] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int c = 0; c < NCH; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[c], 0, 0, 0);
    }
    float s = 0.f;
#pragma unroll
    for (int c = 0; c < NCH; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
    out[(size_t)blockIdx.x * 256 + threadIdx.x] = s;
}

__global__ void __launch_bounds__(256) k_peak_f64(int iters, float scale, float *out) {
    const double a = scale * (double)(threadIdx.x + 1), b = scale * (double)(threadIdx.x + 2);
    f64x4 acc[NCH];
#pragma unroll
    for (int c = 0; c < NCH; ++c) acc[c] = f64x4{0.0, 0.0, 0.0, 0.0};
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int c = 0; c < NCH; ++c) acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[c], 0, 0, 0);
    }
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < NCH; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
    out[(size_t)blockIdx.x * 256 + threadIdx.x] = (float)s;
}

// 16 independent FMA chains per lane (the FP64 FMA's latency is covered by
// the other waves on the SIMD and the chains of this one)
__global__ void __launch_bounds__(256) k_peak_valu64(int iters, float scale, float *out) {
    double x[16];
    const double a = 1.0 + 1e-9 * scale, b = 1e-7 * scale * (double)threadIdx.x;
#pragma unroll
    for (int c = 0; c < 16; ++c) x[c] = scale * (double)(threadIdx.x + c);
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int c = 0; c < 16; ++c) x[c] = fma(x[c], a, b);
    }
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < 16; ++c) s += x[c];
    out[(size_t)blockIdx.x * 256 + threadIdx.x] = (float)s;
}

__global__ void __launch_bounds__(256) k_peak_valu32(int iters, float scale, float *out) {
    float x[16];
    const float a = 1.0f + 1e-6f * scale, b = 1e-5f * scale * (float)threadIdx.x;
#pragma unroll
    for (int c = 0; c < 16; ++c) x[c] = scale * (float)(threadIdx.x + c);
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int c = 0; c < 16; ++c) x[c] = fmaf(x[c], a, b);
    }
    float s = 0.f;
#pragma unroll
    for (int c = 0; c < 16; ++c) s += x[c];
    out[(size_t)blockIdx.x * 256 + threadIdx.x] = s;
}

}  // namespace

extern "C" {

double tnslq_peak_flops_per_round(int kind) {
    switch (kind) {
        case 0: return 16384.0 * NCH;
        case 1: return 2048.0 * NCH;
        case 2: return 2048.0 * NCH;
        case 3: return 2.0 * 64 * 16;
        case 4: return 2.0 * 64 * 16;
        case 5: return 32768.0 * 4;
        default: return 0.0;
    }
}

int tnslq_peak_launch(int kind, int blocks, int iters, float scale, void *out, void *stream) {
    if (blocks < 1 || blocks > (1 << 20) || iters < 1 || !out) return -1;
    hipStream_t st = (hipStream_t)stream;
    float *o = (float *)out;
    switch (kind) {
        case 0: hipLaunchKernelGGL(k_peak_bf16, dim3(blocks), dim3(256), 0, st, iters, scale, o); break;
        case 1: hipLaunchKernelGGL(k_peak_f32, dim3(blocks), dim3(256), 0, st, iters, scale, o); break;
        case 2: hipLaunchKernelGGL(k_peak_f64, dim3(blocks), dim3(256), 0, st, iters, scale, o); break;
        case 3: hipLaunchKernelGGL(k_peak_valu64, dim3(blocks), dim3(256), 0, st, iters, scale, o); break;
        case 4: hipLaunchKernelGGL(k_peak_valu32, dim3(blocks), dim3(256), 0, st, iters, scale, o); break;
        case 5: hipLaunchKernelGGL(k_peak_bf16_32, dim3(blocks), dim3(256), 0, st, iters, scale, o); break;
        default: return -1;
    }
    return hipGetLastError() == hipSuccess ? 0 : -5;
}

}  // extern "C"
