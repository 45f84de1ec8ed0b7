// Operand formats of the two contractions and the contraction launcher
// interface: precisions and their BF16 splits, plane stores, the brick layout
// of an operand, and the GEMM descriptor.  Everything the contraction kernels
// are compiled from, apart from their own source file, is here.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "tnslq.h"

namespace tnslq {

// ------------------------------------------------------------ precisions
// Pieces per real component and bytes per stored piece.
__host__ __device__ constexpr int pieces_of(int prec) {
    return prec == TNSLQ_BF16X6 ? 3 : (prec == TNSLQ_BF16X3 ? 2 : 1);
}
__host__ __device__ constexpr int piece_bytes(int prec) {
    return prec == TNSLQ_FP64 ? 8 : (prec == TNSLQ_FP32 ? 4 : 2);
}
// Planes per stored complex value: the pieces of the real part, then those of
// the imaginary part; split BF16 (BF16X3) also stores the pieces of their sum
// Re + Im, which its contraction needs for the three-product form of a complex
// product (planes re_hi, re_lo, im_hi, im_lo, sum_hi, sum_lo).
__host__ __device__ constexpr int planes_of(int prec) { return prec == TNSLQ_BF16X3 ? 6 : 2 * pieces_of(prec); }

// ------------------------------------------------------------ BF16 helpers
// Round-to-nearest-even FP32 -> BF16 bits (finite inputs; NaN stays NaN).
__device__ inline uint16_t f32_to_bf16_rne(float x) {
    uint32_t u = __float_as_uint(x);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ inline float bf16_to_f32(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

// Split an FP32 value into `np` BF16 pieces whose sum approximates it:
// piece 0 = bf16(x), piece 1 = bf16(x - piece0), piece 2 = bf16(rest).
template <int NP>
__device__ inline void split_bf16(float x, uint16_t *out) {
    float r = x;
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        uint16_t h = f32_to_bf16_rne(r);
        out[p] = h;
        r = r - bf16_to_f32(h);
    }
}
// Split an FP64 value: the first piece is taken from the double directly so
// that the pieces capture the value to ~2^-8 per piece.
template <int NP>
__device__ inline void split_bf16_d(double x, uint16_t *out) {
    double r = x;
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        uint16_t h = f32_to_bf16_rne((float)r);
        out[p] = h;
        r = r - (double)bf16_to_f32(h);
    }
}

// Store one complex value (re, im) into plane arrays at element index `idx`.
// `ps` is the plane stride in elements.  Accepts double inputs.  BF16X3 also
// stores the split of re + im (rounded once, from the inputs' precision).
template <int PREC>
__device__ inline void store_planes(void *base, int64_t ps, int64_t idx, double re, double im) {
    if constexpr (PREC == TNSLQ_FP64) {
        double *p = (double *)base;
        p[idx] = re;
        p[ps + idx] = im;
    } else if constexpr (PREC == TNSLQ_FP32) {
        float *p = (float *)base;
        p[idx] = (float)re;
        p[ps + idx] = (float)im;
    } else {
        constexpr int NP = pieces_of(PREC);
        uint16_t *p = (uint16_t *)base;
        uint16_t h[NP];
        split_bf16_d<NP>(re, h);
#pragma unroll
        for (int q = 0; q < NP; ++q) p[q * ps + idx] = h[q];
        split_bf16_d<NP>(im, h);
#pragma unroll
        for (int q = 0; q < NP; ++q) p[(NP + q) * ps + idx] = h[q];
        if constexpr (PREC == TNSLQ_BF16X3) {
            split_bf16_d<NP>(re + im, h);
#pragma unroll
            for (int q = 0; q < NP; ++q) p[(2 * NP + q) * ps + idx] = h[q];
        }
    }
}
// Same for FP32 accumulator values (the first contraction's output).
template <int PREC>
__device__ inline void store_planes_f(void *base, int64_t ps, int64_t idx, float re, float im) {
    if constexpr (PREC == TNSLQ_FP64) {
        double *p = (double *)base;
        p[idx] = re;
        p[ps + idx] = im;
    } else if constexpr (PREC == TNSLQ_FP32) {
        float *p = (float *)base;
        p[idx] = re;
        p[ps + idx] = im;
    } else {
        constexpr int NP = pieces_of(PREC);
        uint16_t *p = (uint16_t *)base;
        uint16_t h[NP];
        split_bf16<NP>(re, h);
#pragma unroll
        for (int q = 0; q < NP; ++q) p[q * ps + idx] = h[q];
        split_bf16<NP>(im, h);
#pragma unroll
        for (int q = 0; q < NP; ++q) p[(NP + q) * ps + idx] = h[q];
        if constexpr (PREC == TNSLQ_BF16X3) {
            split_bf16<NP>(re + im, h);
#pragma unroll
            for (int q = 0; q < NP; ++q) p[(2 * NP + q) * ps + idx] = h[q];
        }
    }
}

// ------------------------------------------------------------ bricks
// An R x Kr operand is cut into bricks of 128 rows by 64 bytes of the
// reduction index (32 BF16, 16 FP32 or 8 FP64 terms) per plane; a brick holds
// all planes of its piece of the matrix one after the other (8 KiB each, in
// the order of planes_of), and
// bricks run along the reduction index first, then over blocks of 128 rows.
// Within a brick row the four 16-byte units are stored XOR-swizzled by
// ((row >> 1) ^ (row >> 2)) & 3, the order in which the contraction kernel
// keeps them in LDS.  Rows are padded to a multiple of 128 and the reduction
// index to a whole brick; padding along the reduction index must hold zeros.
// One brick is what the contraction kernel stages per reduction step (split
// BF16: one pair of planes at a time), so its loads are contiguous blocks of
// 8 KiB or more.
constexpr int BRICK_ROWS = 128;
constexpr int BRICK_ROW_BYTES = 64;
constexpr int BRICK_PLANE_BYTES = BRICK_ROWS * BRICK_ROW_BYTES;

// reduction terms per brick row
__host__ __device__ constexpr int brick_epr(int prec) { return BRICK_ROW_BYTES / piece_bytes(prec); }
// distance between the planes of one brick, in elements
__host__ __device__ constexpr int64_t brick_ps(int prec) { return (int64_t)BRICK_ROWS * brick_epr(prec); }
// bricks along the reduction index
__host__ __device__ inline int64_t brick_stages(int prec, int64_t Kr) {
    return (Kr + brick_epr(prec) - 1) / brick_epr(prec);
}
__host__ __device__ inline int64_t brick_rows(int64_t R) { return (R + BRICK_ROWS - 1) / BRICK_ROWS * BRICK_ROWS; }
// bytes of one block of 128 rows, and of a whole R x Kr operand
__host__ __device__ inline size_t brick_block_bytes(int prec, int64_t nst) {
    return (size_t)nst * planes_of(prec) * BRICK_PLANE_BYTES;
}
__host__ __device__ inline size_t brick_bytes(int prec, int64_t R, int64_t Kr) {
    return (size_t)(brick_rows(R) / BRICK_ROWS) * brick_block_bytes(prec, brick_stages(prec, Kr));
}
__host__ __device__ inline int brick_swizzle(int64_t row) { return (int)(((row >> 1) ^ (row >> 2)) & 3); }
// Element index (plane 0) of entry (r, l) of an operand with nst bricks along
// the reduction index; plane p of the entry is at + p * brick_ps(prec).
__host__ __device__ inline int64_t brick_index(int prec, int64_t nst, int64_t r, int64_t l) {
    const int epr = brick_epr(prec), epu = epr / 4;
    const int64_t rr = r % BRICK_ROWS, st = l / epr, ll = l % epr;
    const int64_t u = (ll / epu) ^ brick_swizzle(rr);
    return (((r / BRICK_ROWS) * nst + st) * planes_of(prec) * BRICK_ROWS + rr) * epr + u * epu + ll % epu;
}

// ------------------------------------------------------------ GEMM
// C = A * B^T over complex brick operands: A is M x Kr, B is N x Kr, both with
// nst bricks along the reduction index and A, B pointing at their first block
// of rows.  The reduction is split into S equal runs of bricks.  With
// cnb = 2^cnb_log2 and cni = 2^cni_log2, output element (i, j) of split s goes
//   out_mode 0: into a brick operand with c_nst bricks along its reduction
//               index, at row (j / cnb) * crs + i / cni and reduction index
//               (i % cni) * cnb + j % cnb (S = 1);
//   out_mode 1: to interleaved accumulator-type complex values at
//               s * c_split + (j / cnb) * cbs + i * ldc + j % cnb.
struct GemmDesc {
    const void *A;
    const void *B;
    void *C;
    int64_t M, N, Kr, nst;
    int S;
    int out_mode;
    int cnb_log2, cni_log2;
    int64_t crs, c_nst;
    int64_t ldc, cbs, c_split;
};

hipError_t launch_gemm(int prec, const GemmDesc &g, hipStream_t st);
hipError_t launch_gemm_valu(int prec, const GemmDesc &g, hipStream_t st);
bool gemm_mfma_supported(int prec, const GemmDesc &g);
hipError_t launch_gemm_mfma(int prec, const GemmDesc &g, hipStream_t st);

}  // namespace tnslq
