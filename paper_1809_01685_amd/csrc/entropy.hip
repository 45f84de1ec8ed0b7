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
// matrix cores.  Both copies of psi are stored in column panels 512 wide, row
// after row within a panel, and a block owns one panel: a thread owns two
// adjacent columns and walks the rows, so each block streams one contiguous
// region, a wave's load instruction reads 1 KiB (complex64) of one row and
// eight rows' loads are in flight at a time; the entries of up to 8 vectors
// at a row are staged in LDS and broadcast, each read serving two columns
// (more vectors take further passes); products and sums are FP64.  The rows are cut into S
// splits (grid.y) to fill the chip, their partial sums written separately:
// the first pass's partials are added by a small kernel before the second
// pass stages them, the second pass's by the Lanczos kernel that consumes Y.
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

constexpr int CM_THREADS = 256;   // threads per block
constexpr int CM_CPT = 2;         // adjacent columns per thread
constexpr int CM_COLS = CM_THREADS * CM_CPT;   // columns per block = panel width
constexpr int CM_CH = 64;         // rows staged per LDS chunk

// Panel layout of an R x C matrix: column panels of w = min(C, CM_COLS)
// columns, each stored row after row, so that the rows of one block's panel
// are consecutive in memory: element (i, c) at (c / w) R w + i w + c % w.
__device__ inline int64_t panel_index(int64_t i, int64_t c, int64_t R, int64_t C) {
    const int64_t w = C < CM_COLS ? C : CM_COLS;
    return (c / w) * R * w + i * w + c % w;
}

// psi regrouped as an R x C matrix (flat index o = i C + c, bit t of o taken
// from bit map[t] of psi's index), written in panel layout; same dtype.
template <int DTYPE>
__global__ void __launch_bounds__(256) k_regroup(const void *__restrict__ psi, void *__restrict__ out, int64_t R,
                                                 int64_t C, PermDesc pd) {
    const int64_t D = R * C;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; o < D; o += stride) {
        int64_t in = 0;
        for (int t = 0; t < pd.L; ++t) in |= ((o >> t) & 1) << pd.map[t];
        const int64_t dst = panel_index(o / C, o % C, R, C);
        if constexpr (DTYPE == TNSLQ_C128)
            ((double2 *)out)[dst] = ((const double2 *)psi)[in];
        else
            ((float2 *)out)[dst] = ((const float2 *)psi)[in];
    }
}

// The two adjacent elements (i, c), (i, c + 1) at panel offset e of M.
template <int DTYPE>
__device__ inline void load_pair(const void *M, int64_t e, double2 &a, double2 &b) {
    if constexpr (DTYPE == TNSLQ_C128) {
        a = ((const double2 *)M)[e];
        b = ((const double2 *)M)[e + 1];
    } else {
        const float4 f = *(const float4 *)((const float2 *)M + e);
        a = make_double2(f.x, f.y);
        b = make_double2(f.z, f.w);
    }
}

// out[s][k][c] = sum over rows i of split s of op(M[i][c]) V[k][i] for the KG
// vectors k0 = blockIdx.z KG ..; op = conj if CONJ; M in panel layout, block x
// owning panel x, thread t its columns 2t, 2t + 1.  The vector entries of a
// row are staged in LDS and broadcast; each serves two columns.
template <int DTYPE, bool CONJ, int KG>
__global__ void __launch_bounds__(CM_THREADS) k_colmac(const void *__restrict__ M, int64_t R, int64_t C,
                                                       const double2 *__restrict__ V, int K,
                                                       double2 *__restrict__ out, int64_t out_split_stride,
                                                       int64_t rows_per_split) {
    constexpr int U = 8;   // rows whose loads are issued together
    __shared__ double2 vs[KG][CM_CH];
    const int t = threadIdx.x;
    const int64_t c = ((int64_t)blockIdx.x * CM_THREADS + t) * CM_CPT;
    const int s = blockIdx.y;
    const int kg0 = blockIdx.z * KG;
    const int kn = K - kg0 < KG ? K - kg0 : KG;
    const int64_t i0 = (int64_t)s * rows_per_split;
    const int64_t i1 = i0 + rows_per_split < R ? i0 + rows_per_split : R;
    const int64_t w = C < CM_COLS ? C : CM_COLS;
    double ar[CM_CPT][KG], ai[CM_CPT][KG];
#pragma unroll
    for (int j = 0; j < CM_CPT; ++j)
#pragma unroll
        for (int k = 0; k < KG; ++k) ar[j][k] = ai[j][k] = 0.0;
    for (int64_t ib = i0; ib < i1; ib += CM_CH) {
        const int nrow = (int)(i1 - ib < CM_CH ? i1 - ib : CM_CH);
        __syncthreads();
        for (int e = t; e < KG * CM_CH; e += CM_THREADS) {
            const int k = e / CM_CH, ii = e % CM_CH;
            vs[k][ii] = (k < kn && ii < nrow) ? V[(int64_t)(kg0 + k) * R + ib + ii] : make_double2(0.0, 0.0);
        }
        __syncthreads();
        if (c < C) {
            const int64_t base = panel_index(ib, c, R, C);
            for (int u0 = 0; u0 < nrow; u0 += U) {
                // the U row loads of a batch are issued before any is used
                double2 ma[U], mb[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    if (u0 + u < nrow) {
                        load_pair<DTYPE>(M, base + (int64_t)(u0 + u) * w, ma[u], mb[u]);
                    } else {
                        ma[u] = make_double2(0.0, 0.0);
                        mb[u] = ma[u];
                    }
                }
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const double ax = ma[u].x, ay = CONJ ? -ma[u].y : ma[u].y;
                    const double bx = mb[u].x, by = CONJ ? -mb[u].y : mb[u].y;
#pragma unroll
                    for (int k = 0; k < KG; ++k) {
                        const double2 v = vs[k][(u0 + u) & (CM_CH - 1)];
                        ar[0][k] = fma(ax, v.x, fma(-ay, v.y, ar[0][k]));
                        ai[0][k] = fma(ax, v.y, fma(ay, v.x, ai[0][k]));
                        ar[1][k] = fma(bx, v.x, fma(-by, v.y, ar[1][k]));
                        ai[1][k] = fma(bx, v.y, fma(by, v.x, ai[1][k]));
                    }
                }
            }
        }
    }
    if (c < C) {
#pragma unroll
        for (int k = 0; k < KG; ++k)
            if (k < kn) {
                double2 *o = out + s * out_split_stride + (int64_t)(kg0 + k) * C + c;
                o[0] = make_double2(ar[0][k], ai[0][k]);
                o[1] = make_double2(ar[1][k], ai[1][k]);
            }
    }
}

// Z[k][i] = sum_s Zp[s][k][i], n = K x n_i elements.
__global__ void __launch_bounds__(256) k_sum_splits(const double2 *__restrict__ part, int S, int64_t n,
                                                    double2 *__restrict__ Z) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) {
        double x = 0.0, y = 0.0;
        for (int p = 0; p < S; ++p) {
            const double2 v = part[p * n + e];
            x += v.x;
            y += v.y;
        }
        Z[e] = make_double2(x, y);
    }
}

}  // namespace

hipError_t launch_regroup(int dtype, const void *psi, void *out, int64_t R, int64_t C, const PermDesc &pd,
                          hipStream_t st) {
    int64_t g = (R * C + 1023) / 1024;
    if (g < 1) g = 1;
    if (g > 65535 * 8) g = 65535 * 8;
    if (dtype == TNSLQ_C128)
        hipLaunchKernelGGL((k_regroup<TNSLQ_C128>), dim3((unsigned)g), dim3(256), 0, st, psi, out, R, C, pd);
    else
        hipLaunchKernelGGL((k_regroup<TNSLQ_C64>), dim3((unsigned)g), dim3(256), 0, st, psi, out, R, C, pd);
    return hipGetLastError();
}

template <int KG>
void colmac_kg(int dtype, int conj, dim3 grid, hipStream_t st, const void *M, int64_t R, int64_t C,
               const double2 *V, int K, double2 *out, int64_t ostride, int64_t rps) {
#define TNSLQ_CM(T, CJ) \
    hipLaunchKernelGGL((k_colmac<T, CJ, KG>), grid, dim3(CM_THREADS), 0, st, M, R, C, V, K, out, ostride, rps)
    if (dtype == TNSLQ_C128) {
        if (conj) TNSLQ_CM(TNSLQ_C128, true);
        else TNSLQ_CM(TNSLQ_C128, false);
    } else {
        if (conj) TNSLQ_CM(TNSLQ_C64, true);
        else TNSLQ_CM(TNSLQ_C64, false);
    }
#undef TNSLQ_CM
}

hipError_t launch_colmac(int dtype, int conj, const void *M, int64_t R, int64_t C, const double2 *V, int K,
                         double2 *out, int S, hipStream_t st) {
    if (R < 1 || C < 1 || K < 1 || S < 1 || R % S != 0) return hipErrorInvalidValue;
    // vectors per pass over M: the smallest of 1, 2, 4, 8 covering K (8 and
    // several passes beyond: 16 would leave one wave per SIMD)
    const int kg = K <= 1 ? 1 : K <= 2 ? 2 : K <= 4 ? 4 : 8;
    if (C % CM_CPT != 0) return hipErrorInvalidValue;
    const int64_t gx = (C + CM_COLS - 1) / CM_COLS, gz = (K + kg - 1) / kg;
    if (gx > 0x7fffffff || S > 65535 || gz > 65535) return hipErrorInvalidConfiguration;
    const dim3 grid((unsigned)gx, (unsigned)S, (unsigned)gz);
    const int64_t rps = R / S, ostride = (int64_t)K * C;
    switch (kg) {
        case 1: colmac_kg<1>(dtype, conj, grid, st, M, R, C, V, K, out, ostride, rps); break;
        case 2: colmac_kg<2>(dtype, conj, grid, st, M, R, C, V, K, out, ostride, rps); break;
        case 4: colmac_kg<4>(dtype, conj, grid, st, M, R, C, V, K, out, ostride, rps); break;
        default: colmac_kg<8>(dtype, conj, grid, st, M, R, C, V, K, out, ostride, rps); break;
    }
    return hipGetLastError();
}

hipError_t launch_sum_splits(const double2 *part, int S, int64_t n, double2 *Z, hipStream_t st) {
    int64_t g = (n + 255) / 256;
    if (g > 65535 * 4) g = 65535 * 4;
    if (g < 1) g = 1;
    hipLaunchKernelGGL(k_sum_splits, dim3((unsigned)g), dim3(256), 0, st, part, S, n, Z);
    return hipGetLastError();
}

}  // namespace tnslq
