// Internal declarations shared by the libtnslq translation units.
//
// Data layout in HBM.  The four operands of the two contractions are complex
// matrices of R rows by Kr reduction terms, stored in bricks (below):
//   P_aeb   psi regrouped as (A, E, B): d_A rows a, reduction index (c, b')
//           (b' fastest) of the second contraction.
//   P_bea   psi regrouped as (B, E, A) and conjugated: d_B d_E rows (b, c),
//           reduction index a' of the first contraction.
//   Xt      the current Lanczos vectors: rows (k, b'), reduction index a'.
//   Ups     intermediary (i) of Sec. V: rows (k, b), reduction index (c, b'),
//           the B operand of the second contraction.
//   Ypart   FP32 or FP64 split-K partial sums of Y[k][a][b], interleaved
//           complex, row-major.
// Both contractions are therefore "NT" products C = A * B^T whose operands are
// bricked along the reduction index.
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
__host__ __device__ constexpr int planes_of(int prec) { return 2 * pieces_of(prec); }

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
// `ps` is the plane stride in elements.  Accepts double inputs.
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
    }
}

// ------------------------------------------------------------ plan
struct Plan {
    int L = 0;
    int nA = 0, nB = 0, nE = 0;      // sizes in the roles used on the device
    int qa[TNSLQ_MAX_QUBITS], qb[TNSLQ_MAX_QUBITS], qe[TNSLQ_MAX_QUBITS];
    int swapped = 0;                 // roles of A and B exchanged
    int64_t dA = 1, dB = 1, dE = 1, dAB = 1, D = 1;
    int dtype = TNSLQ_C64;
    int prec = TNSLQ_FP32;
    int K = 1, m = 1, reorth = 0;
    int kc = 1;                      // probes per contraction chunk
    int S = 1;                       // split-K factor of the second contraction
    int nblk = 1;                    // reduction blocks per probe vector
    int64_t nst1 = 1, nst2 = 1;      // bricks along the reduction index of contraction 1, 2
    // workspace carve-up (byte offsets)
    size_t off_Paeb = 0, off_Pbea = 0, off_Xt = 0, off_Ups = 0, off_Ypart = 0;
    size_t off_Q = 0, off_w = 0, off_alpha = 0, off_beta = 0, off_F = 0, off_G = 0;
    size_t off_stats = 0, off_red = 0, off_h = 0, off_steps = 0, off_feat = 0, off_mlp = 0;
    size_t total = 0;
    int nQ = 3;                      // Lanczos vector slots
};

// ------------------------------------------------------------ bricks
// An R x Kr operand is cut into bricks of 128 rows by 64 bytes of the
// reduction index (32 BF16, 16 FP32 or 8 FP64 terms) per plane; a brick holds
// all planes of its piece of the matrix one after the other (8 KiB each), and
// bricks run along the reduction index first, then over blocks of 128 rows.
// Within a brick row the four 16-byte units are stored XOR-swizzled by
// ((row >> 1) ^ (row >> 2)) & 3, the order in which the contraction kernel
// keeps them in LDS.  Rows are padded to a multiple of 128 and the reduction
// index to a whole brick; padding along the reduction index must hold zeros.
// One brick is what the contraction kernel stages per reduction step, so its
// loads are contiguous 8 KiB blocks.
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

// ------------------------------------------------------------ layout
struct PermDesc {
    int L;
    int map[TNSLQ_MAX_QUBITS];   // output bit t <- input bit map[t]
};
// Regroup psi into an R x Kr brick operand (output flat index r * Kr + l),
// writing every brick entry including the zero padding.
hipError_t launch_permute(int prec, int dtype, const void *psi, void *out, int64_t R, int64_t Kr,
                          const PermDesc &pd, int conj, hipStream_t st);

// ------------------------------------------------------------ Lanczos etc.
struct LzDims {
    int64_t dA, dB, n;   // n = dA * dB per probe
    int K, m, nblk;
};
// Xt arguments below are the brick operand of K d_B rows (k, b') by d_A
// reduction terms a', with xt_nst = brick_stages(prec, d_A).
hipError_t launch_probe_init(int prec, const LzDims &z, uint64_t seed, uint64_t offset, int swapped,
                             double2 *q, void *Xt, int64_t xt_nst, double *alpha, double *beta,
                             hipStream_t st);
hipError_t launch_passA(int accfp64, const LzDims &z, const void *part, int S, int64_t split_stride,
                        int k0, int kc, const double2 *q_prev, const double2 *q_cur, double2 *w,
                        const double *alpha, const double *beta, int j, double *dotpart,
                        hipStream_t st);
hipError_t launch_passB(const LzDims &z, const double *dotpart, const double2 *q_cur, double2 *w,
                        double *alpha, const double *beta, int j, double *nrmpart, int want_norm,
                        hipStream_t st);
hipError_t launch_reorth(const LzDims &z, const double2 *Q, int nvec, int64_t q_slot_stride,
                         double2 *w, double *hpart, double2 *h, const double *alpha,
                         const double *beta, int j, double *nrmpart, hipStream_t st);
hipError_t launch_passC(int prec, const LzDims &z, const double *nrmpart, const double2 *w,
                        double2 *q_next, void *Xt, int64_t xt_nst, const double *alpha,
                        double *beta, int j, hipStream_t st);
hipError_t launch_quadrature(const double *alpha, const double *beta, const int *steps, int K,
                             int m, int jlo, int jhi, double *F, hipStream_t st);
hipError_t launch_steps(const double *alpha, const double *beta, int K, int m, int jdone,
                        int *steps, hipStream_t st);
hipError_t launch_stats(const double *beta, const double *F, int K, int m, int j, double *G,
                        double *stats, hipStream_t st);
hipError_t launch_reduce_partials(int accfp64, const void *part, int S, int64_t split_stride,
                                  int64_t dA, int64_t dB, int K, int swapped, double2 *Y,
                                  hipStream_t st);
hipError_t launch_probes_plain(uint64_t seed, uint64_t offset, int K, int64_t d, double2 *X,
                               hipStream_t st);
hipError_t launch_load_vectors(int prec, const double2 *X, int64_t dA, int64_t dB, int K,
                               int swapped, void *Xt, int64_t xt_nst, hipStream_t st);
hipError_t launch_features(const double *alpha, const double *beta, int K, int m, int n_early,
                           double dAB, double dA, double dB, double dE, float *feat,
                           hipStream_t st);

// ------------------------------------------------------------ MLP
size_t mlp_ws_bytes(int batch);
hipError_t mlp_forward(const float *params, const float *norm, const float *x, int batch, float *out,
                       void *ws, hipStream_t st);
hipError_t mlp_loss_grad(const float *params, const float *norm, const float *x, const float *r,
                         const int *idx, int batch, float *loss, float *grad, void *ws,
                         hipStream_t st);
hipError_t mlp_adam(float *params, float *m, float *v, const float *grad, int n, int t, float lr,
                    hipStream_t st);

}  // namespace tnslq
