// The reduced density matrix of a subsystem applied lazily, for the other
// spectral sums of the method (von Neumann entropy, purity): the paper's
// closing section drops the partial transpose and keeps Algorithm 1.
//
// With Psi = psi regrouped as a d x d_R matrix (d the side the Krylov space
// lives on), rho X = Psi (Psi^dagger X) is two passes over psi:
//   Z[k][r] = sum_s conj(Psi[s][r]) X[k][s]   over P1 = Psi   (d x d_R)
//   Y[k][s] = sum_r Psi^T[r][s] Z[k][r]        over P2 = Psi^T (d_R x d)
// both "column MACs" out[k][c] = sum_i op(M[i][c]) V[k][i] over a row-major
// R x C matrix M.  There are only K columns of X, so the passes do K complex
// multiply-adds per element of psi read: they are bound by HBM, not by the
// matrix cores.  A thread owns one column c and walks the rows, so every load
// instruction of a wave reads consecutive elements of one row; the K vector
// entries of a row are broadcast from LDS; products and sums are FP64.  The
// rows are cut into S splits (grid.y) to fill the chip, their partial sums
// written separately: the first pass's partials are added while the second
// stages them, the second pass's by the Lanczos kernel that consumes Y.
#include "tnslq_internal.h"

namespace tnslq {
namespace {

template <int DTYPE>
__device__ inline double2 load_c(const void *p, int64_t i) {
    if constexpr (DTYPE == TNSLQ_C128) {
        return ((const double2 *)p)[i];
    } else {
        const float2 v = ((const float2 *)p)[i];
        return make_double2(v.x, v.y);
    }
}

// out[o] = psi[in(o)], bit t of o taken from bit map[t] of in; same dtype.
template <int DTYPE>
__global__ void __launch_bounds__(256) k_regroup(const void *__restrict__ psi, void *__restrict__ out, int64_t D,
                                                 PermDesc pd) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; o < D; o += stride) {
        int64_t in = 0;
        for (int t = 0; t < pd.L; ++t) in |= ((o >> t) & 1) << pd.map[t];
        if constexpr (DTYPE == TNSLQ_C128)
            ((double2 *)out)[o] = ((const double2 *)psi)[in];
        else
            ((float2 *)out)[o] = ((const float2 *)psi)[in];
    }
}

constexpr int CM_THREADS = 256;   // columns per block
constexpr int CM_KG = 8;          // vectors per pass (grid.z covers more)
constexpr int CM_CH = 64;         // rows staged per LDS chunk

// out[s][k][c] = sum over rows i of split s of op(M[i][c]) V[k][i], op = conj
// if CONJ; V[k][i] = sum_p V[p][k][i] over v_splits partial arrays.
template <int DTYPE, bool CONJ>
__global__ void __launch_bounds__(CM_THREADS) k_colmac(const void *__restrict__ M, int64_t R, int64_t C,
                                                       const double2 *__restrict__ V, int v_splits,
                                                       int64_t v_split_stride, int K, double2 *__restrict__ out,
                                                       int64_t out_split_stride, int64_t rows_per_split) {
    __shared__ double2 vs[CM_KG][CM_CH];
    const int t = threadIdx.x;
    const int64_t c = (int64_t)blockIdx.x * CM_THREADS + t;
    const int s = blockIdx.y;
    const int kg0 = blockIdx.z * CM_KG;
    const int kn = K - kg0 < CM_KG ? K - kg0 : CM_KG;
    const int64_t i0 = (int64_t)s * rows_per_split;
    const int64_t i1 = i0 + rows_per_split < R ? i0 + rows_per_split : R;
    double ar[CM_KG], ai[CM_KG];
#pragma unroll
    for (int k = 0; k < CM_KG; ++k) ar[k] = ai[k] = 0.0;
    for (int64_t ib = i0; ib < i1; ib += CM_CH) {
        const int nrow = (int)(i1 - ib < CM_CH ? i1 - ib : CM_CH);
        __syncthreads();
        for (int e = t; e < CM_KG * CM_CH; e += CM_THREADS) {
            const int k = e / CM_CH, ii = e % CM_CH;
            double2 v = make_double2(0.0, 0.0);
            if (k < kn && ii < nrow) {
                for (int p = 0; p < v_splits; ++p) {
                    const double2 u = V[p * v_split_stride + (int64_t)(kg0 + k) * R + ib + ii];
                    v.x += u.x;
                    v.y += u.y;
                }
            }
            vs[k][ii] = v;
        }
        __syncthreads();
        if (c < C) {
            const int64_t base = ib * C + c;
#pragma unroll 4
            for (int ii = 0; ii < nrow; ++ii) {
                double2 m = load_c<DTYPE>(M, base + (int64_t)ii * C);
                if constexpr (CONJ) m.y = -m.y;
#pragma unroll
                for (int k = 0; k < CM_KG; ++k) {
                    const double2 v = vs[k][ii];
                    ar[k] = fma(m.x, v.x, fma(-m.y, v.y, ar[k]));
                    ai[k] = fma(m.x, v.y, fma(m.y, v.x, ai[k]));
                }
            }
        }
    }
    if (c < C) {
#pragma unroll
        for (int k = 0; k < CM_KG; ++k)
            if (k < kn) out[s * out_split_stride + (int64_t)(kg0 + k) * C + c] = make_double2(ar[k], ai[k]);
    }
}

}  // namespace

hipError_t launch_regroup(int dtype, const void *psi, void *out, int64_t D, const PermDesc &pd, hipStream_t st) {
    int64_t g = (D + 1023) / 1024;
    if (g < 1) g = 1;
    if (g > 65535 * 8) g = 65535 * 8;
    if (dtype == TNSLQ_C128)
        hipLaunchKernelGGL((k_regroup<TNSLQ_C128>), dim3((unsigned)g), dim3(256), 0, st, psi, out, D, pd);
    else
        hipLaunchKernelGGL((k_regroup<TNSLQ_C64>), dim3((unsigned)g), dim3(256), 0, st, psi, out, D, pd);
    return hipGetLastError();
}

hipError_t launch_colmac(int dtype, int conj, const void *M, int64_t R, int64_t C, const double2 *V, int v_splits,
                         int64_t v_split_stride, int K, double2 *out, int S, hipStream_t st) {
    if (R < 1 || C < 1 || K < 1 || S < 1 || R % S != 0) return hipErrorInvalidValue;
    const int64_t gx = (C + CM_THREADS - 1) / CM_THREADS, gz = (K + CM_KG - 1) / CM_KG;
    if (gx > 0x7fffffff || S > 65535 || gz > 65535) return hipErrorInvalidConfiguration;
    dim3 grid((unsigned)gx, (unsigned)S, (unsigned)gz), block(CM_THREADS);
    const int64_t rps = R / S, ostride = (int64_t)K * C;
#define TNSLQ_CM(T, CJ) \
    hipLaunchKernelGGL((k_colmac<T, CJ>), grid, block, 0, st, M, R, C, V, v_splits, v_split_stride, K, out, ostride, rps)
    if (dtype == TNSLQ_C128) {
        if (conj) TNSLQ_CM(TNSLQ_C128, true);
        else TNSLQ_CM(TNSLQ_C128, false);
    } else {
        if (conj) TNSLQ_CM(TNSLQ_C64, true);
        else TNSLQ_CM(TNSLQ_C64, false);
    }
#undef TNSLQ_CM
    return hipGetLastError();
}

}  // namespace tnslq
