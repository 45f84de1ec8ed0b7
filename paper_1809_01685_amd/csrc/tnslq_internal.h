// Internal declarations shared by the libtnslq translation units.
//
// Data layout in HBM (all complex operands of the contractions are stored as
// separate planes, one real array per component piece):
//   P_aeb   psi regrouped as (A, E, B), b fastest: a d_A x (d_E d_B) matrix.
//           Row a holds psi[a, c, b'] over the reduction index (c, b') of the
//           second contraction.
//   P_bea   psi regrouped as (B, E, A), a fastest and conjugated: a
//           (d_B d_E) x d_A matrix whose rows (b, c) hold conj psi[a', b, c]
//           over the reduction index a' of the first contraction.
//   Xt      the current Lanczos vectors, transposed to [k][b'][a'] (a' fastest).
//   Ups     intermediary (i) of Sec. V, Ups[k][(b, c)][b'], which read as
//           [k][b][(c, b')] is the B operand of the second contraction.
//   Ypart   FP32 or FP64 split-K partial sums of Y[k][a][b].
// Both contractions are therefore "NT" products C = A * B^T in which both
// operands are contiguous along the reduction index.
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

// Plane stride in elements for an array of n complex elements (256-byte
// aligned planes for every piece size).
__host__ __device__ inline int64_t plane_stride(int64_t n) { return (n + 127) / 128 * 128; }

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
    // workspace carve-up (byte offsets)
    size_t off_Paeb = 0, off_Pbea = 0, off_Xt = 0, off_Ups = 0, off_Ypart = 0;
    size_t off_Q = 0, off_w = 0, off_alpha = 0, off_beta = 0, off_F = 0, off_G = 0;
    size_t off_stats = 0, off_red = 0, off_h = 0, off_steps = 0, off_feat = 0, off_mlp = 0;
    size_t total = 0;
    int nQ = 3;                      // Lanczos vector slots
};

// ------------------------------------------------------------ GEMM
// C = A * B^T over complex planes; A is M x Kr (row stride lda), B is N x Kr
// (row stride ldb), both contiguous along the reduction index.  Output
// element (i, j) goes to (j / cnb) * cbs + i * ldc + (j % cnb), either as
// low-precision planes (out_mode 0) or as interleaved accumulator-type
// complex values of split s at offset s * c_split (out_mode 1).
struct GemmDesc {
    const void *A;
    int64_t lda, a_ps;
    const void *B;
    int64_t ldb, b_ps;
    void *C;
    int64_t c_ps;
    int64_t M, N, Kr;
    int64_t ldc, cnb, cbs;
    int S;
    int64_t c_split;
    int out_mode;
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
hipError_t launch_permute(int prec, int dtype, const void *psi, void *out, int64_t ps, int64_t D,
                          const PermDesc &pd, int conj, hipStream_t st);

// ------------------------------------------------------------ Lanczos etc.
struct LzDims {
    int64_t dA, dB, n;   // n = dA * dB per probe
    int K, m, nblk;
};
hipError_t launch_probe_init(int prec, const LzDims &z, uint64_t seed, uint64_t offset, int swapped,
                             double2 *q, void *Xt, int64_t xt_ps, double *alpha, double *beta,
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
                        double2 *q_next, void *Xt, int64_t xt_ps, const double *alpha,
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
                               int swapped, void *Xt, int64_t xt_ps, hipStream_t st);
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
