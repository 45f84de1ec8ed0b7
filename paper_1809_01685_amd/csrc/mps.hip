// Contiguous blocks of a matrix product state, open or periodic (Sec. VI):
// the compressed form of rho_AB^{T_B}, as two factors P, Q of an effective
// state whose partially transposed density matrix has the same nonzero
// spectrum (applied in factorised form, or contracted into that state).
//
// All of it is FP64 linear algebra on tensors of bond dimension chi:
//   * transfer sweeps for the traced environments left of A and right of B
//     of an open chain, E <- sum_s M_s^T E conj(M_s) (two complex products
//     per site);
//   * transfer matrices of whole sections, T[(x, x')][y'][y] (chi^4 entries),
//     one site at a time (one complex product and chi^2 small batched ones per
//     site), for blocks, gaps and the ring's outer section of any length:
//     the Gram matrix of a block and the factored matrix of a traced section
//     are T with its four axes regrouped;
//   * Cholesky factors of positive semidefinite matrices (environments, Gram
//     matrices of the blocks, of the gap and of a ring's outer section),
//     blocked: panels of 32 columns in one workgroup, the solve below them
//     and the trailing update across the GPU;
//   * complex matrix products C = op(A) op(B), batched, op in {N, T, C}
//     (64 x 64 output tiles staged through LDS, FP64 matrix instructions),
//     for the block sections, their Gram matrices, the effective state and
//     the factorised operator;
//   * the factor normalisation Re sum Ahat conj(C);
//   * axis exchanges and permutations, and the final scatter of the effective
//     state into a zero-padded power-of-two layout, normalised.
// The host side (api.hip) plans the sizes and sequences these launches.
#include "tnslq_internal.h"

namespace tnslq {
namespace {

__device__ inline double2 cmul(double2 a, double2 b) { return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
__device__ inline double2 cconj(double2 a) { return make_double2(a.x, -a.y); }

// Normalise a small positive matrix by its trace (one block): keeps long
// sweeps in range; the effective state is normalised at the end.
__global__ void __launch_bounds__(256) k_scale_by_trace(double2 *__restrict__ E, int n) {
    __shared__ double tr;
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int i = 0; i < n; ++i) s += E[i * n + i].x;
        tr = s > 0.0 ? s : 1.0;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < n * n; i += blockDim.x) E[i] = make_double2(E[i].x / tr, E[i].y / tr);
}

// In-place lower Cholesky factor of a Hermitian positive semidefinite n x n
// matrix (row-major): A = L L^dagger, L lower triangular with a real
// non-negative diagonal; the strict upper triangle is zeroed.  A pivot not
// above 1e-13 of the largest diagonal entry of the input (the matrix is rank
// deficient there; Gram and transfer matrices are positive semidefinite by
// construction) leaves its column zero: L L^dagger is still the matrix, and
// the zero columns only add zero padding downstream.  *fail is set when a
// pivot is not finite (and never cleared here).
//
// Blocked, right-looking, in panels of CNB columns: the diagonal block is
// factored in one workgroup (k_chol_panel), the rows below solve against it
// (k_chol_trsm), and the trailing matrix takes the rank-CNB update
// A22 -= L21 L21^dagger as a complex product (k_zgemm, subtracting).
constexpr int CNB = 32;

__global__ void __launch_bounds__(256) k_chol_init(const double2 *__restrict__ A, int n, double *__restrict__ dmax) {
    __shared__ double sh[256];
    double m = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) m = fmax(m, A[(int64_t)i * n + i].x);
    sh[threadIdx.x] = m;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) *dmax = sh[0];
}

// Factor the w x w diagonal block at (j0, j0), w = min(CNB, n - j0), whose
// entries already hold every update from the columns before j0.
__global__ void __launch_bounds__(256) k_chol_panel(double2 *__restrict__ A, int n, int j0,
                                                    const double *__restrict__ dmax, int *__restrict__ fail) {
    __shared__ double2 T[CNB][CNB + 1];
    const int w = min(CNB, n - j0);
    for (int e = threadIdx.x; e < CNB * CNB; e += 256) {
        const int r = e / CNB, c = e % CNB;
        T[r][c] = (r < w && c <= r) ? A[(int64_t)(j0 + r) * n + j0 + c] : make_double2(0.0, 0.0);
    }
    const double tol = 1e-13 * *dmax;
    __syncthreads();
    for (int j = 0; j < w; ++j) {
        if (threadIdx.x == 0) {
            const double d = T[j][j].x;
            if (!isfinite(d)) *fail = 1;
            T[j][j] = make_double2(d > tol ? sqrt(d) : 0.0, 0.0);
        }
        __syncthreads();
        const double piv = T[j][j].x;
        for (int i = j + 1 + threadIdx.x; i < w; i += 256)
            T[i][j] = piv > 0.0 ? make_double2(T[i][j].x / piv, T[i][j].y / piv) : make_double2(0.0, 0.0);
        __syncthreads();
        // rank-1 update of the block's remaining lower triangle
        const int m = w - j - 1;
        for (int e = threadIdx.x; e < m * m; e += 256) {
            const int i = j + 1 + e / m, k = j + 1 + e % m;
            if (k <= i) {
                const double2 q = cmul(T[i][j], cconj(T[k][j]));
                T[i][k] = make_double2(T[i][k].x - q.x, T[i][k].y - q.y);
            }
        }
        __syncthreads();
    }
    for (int e = threadIdx.x; e < w * w; e += 256) {
        const int r = e / w, c = e % w;
        if (c <= r) A[(int64_t)(j0 + r) * n + j0 + c] = T[r][c];
    }
}

// Rows r >= j0 + w: L21[r][:] solves x L11^dagger = A[r][j0 .. j0 + w), one
// row per thread (zero pivots give zero entries, as in the unblocked form).
__global__ void __launch_bounds__(256) k_chol_trsm(double2 *__restrict__ A, int n, int j0) {
    __shared__ double2 L[CNB][CNB + 1];
    const int w = min(CNB, n - j0);
    for (int e = threadIdx.x; e < CNB * CNB; e += 256) {
        const int r = e / CNB, c = e % CNB;
        L[r][c] = (r < w && c <= r) ? A[(int64_t)(j0 + r) * n + j0 + c] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    const int64_t r = (int64_t)j0 + w + (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (r >= n) return;
    double2 *row = A + r * n + j0;
    double2 x[CNB];
#pragma unroll
    for (int k = 0; k < CNB; ++k) {
        if (k < w) {
            double2 v = row[k];
#pragma unroll
            for (int m = 0; m < k; ++m) {
                const double2 q = cmul(x[m], cconj(L[k][m]));
                v = make_double2(v.x - q.x, v.y - q.y);
            }
            const double piv = L[k][k].x;
            x[k] = piv > 0.0 ? make_double2(v.x / piv, v.y / piv) : make_double2(0.0, 0.0);
            row[k] = x[k];
        } else {
            x[k] = make_double2(0.0, 0.0);
        }
    }
}

__global__ void __launch_bounds__(256) k_zero_upper(double2 *__restrict__ A, int n) {
    const int64_t total = (int64_t)n * n;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x)
        if (e % n > e / n) A[e] = make_double2(0.0, 0.0);
}

// C[b] = op(A[b]) op(B[b]) (C[b] -= op(A[b]) op(B[b]) with sub) for complex
// row-major matrices, in FP64 (double2) or FP32 (float2): op(A) is M x K,
// op(B) is K x N; OP = 0 (as stored), 1 (transpose), 2 (conjugate transpose);
// lda/ldb/ldc are the stored row strides, sa/sb/sc the batch strides.  A
// block of 256 threads (4 waves) computes a 64 x 64 tile, staging 64 x 16
// slices of op(A) and 16 x 64 of op(B) through LDS (zeros outside the
// matrices; each step's slices are loaded into registers during the
// previous step's products); each wave owns 32 x 32 outputs as 2 x 2 tiles of
// v_mfma_f64_16x16x4f64 (v_mfma_f32_16x16x4f32), four real products per
// complex one (Cr += Ar Br - Ai Bi, Ci += Ar Bi + Ai Br).  Lane l supplies
// A[l % 16][k] and B[k][l % 16] with k = l / 16 of each 4-term step; its
// accumulator register r holds output row 4 r + l / 16 (FP64) or
// 4 (l / 16) + r (FP32), column l % 16.
typedef __attribute__((ext_vector_type(4))) double f64x4;
typedef __attribute__((ext_vector_type(4))) float f32x4;

template <typename T> struct ZT;
template <> struct ZT<double> {
    using C2 = double2;
    using V = f64x4;
    static __device__ V mfma(double a, double b, V c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
    static __device__ int row(int r, int fk) { return 4 * r + fk; }
};
template <> struct ZT<float> {
    using C2 = float2;
    using V = f32x4;
    static __device__ V mfma(float a, float b, V c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
    static __device__ int row(int r, int fk) { return 4 * fk + r; }
};

// XC: output (r, c) with r = (r1, r2), r2 < xm, and c = (c1, c2), c2 < xv,
// lands at ((r1 xm + c1) xm + r2) xv + c2 of its batch entry, i.e. the
// result with r2 and c1 exchanged (ldc unused).
template <int OPA, int OPB, typename T, bool XC = false>
__global__ void __launch_bounds__(256) k_zgemm(const typename ZT<T>::C2 *__restrict__ A,
                                               const typename ZT<T>::C2 *__restrict__ B,
                                               typename ZT<T>::C2 *__restrict__ C, int M, int N, int K, int64_t lda,
                                               int64_t ldb, int64_t ldc, int64_t sa, int64_t sb, int64_t sc,
                                               int sub, int ks, int64_t csk, int64_t xm = 1, int64_t xv = 1) {
    using C2 = typename ZT<T>::C2;
    using V = typename ZT<T>::V;
    constexpr int TM = 64, TN = 64, TK = 16;
    __shared__ C2 As[TK][TM + 1], Bs[TK][TN + 1];
    // grid z = (batch entry b, reduction split s): split s sums terms
    // [kbeg, kend) into C + b sc + s csk
    const int64_t b = blockIdx.z / ks;
    const int sp = (int)(blockIdx.z % ks);
    const int Kc = ((K + ks - 1) / ks + TK - 1) / TK * TK;
    const int kbeg = sp * Kc, kend = min(K, kbeg + Kc);
    A += b * sa;
    B += b * sb;
    C += b * sc + sp * csk;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6, wm = w >> 1, wn = w & 1;
    const int fr = lane & 15, fk = lane >> 4;
    const int r0 = blockIdx.y * TM, c0 = blockIdx.x * TN;
    V accr[2][2], acci[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            accr[i][j] = V{0, 0, 0, 0};
            acci[i][j] = V{0, 0, 0, 0};
        }
    // The slices of k0 + TK are loaded into registers while the MFMAs of k0
    // run (their global latency hidden behind the arithmetic), then stored
    // to LDS between the two barriers of the next step.
    C2 ra[4], rb[4];
    auto load = [&](int k0) {
        // 1024 entries of each slice, four per thread
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int e = t + 256 * q;
            {
                // op(A)[r0 + rr][k0 + kk]
                const int rr = OPA == 0 ? e / TK : e % TM, kk = OPA == 0 ? e % TK : e / TM;
                const int r = r0 + rr, k = k0 + kk;
                C2 v = {0, 0};
                if (r < M && k < kend) {
                    v = OPA == 0 ? A[(int64_t)r * lda + k] : A[(int64_t)k * lda + r];
                    if (OPA == 2) v.y = -v.y;
                }
                ra[q] = v;
            }
            {
                // op(B)[k0 + kk][c0 + cc]
                const int cc = OPB == 0 ? e % TN : e / TK, kk = OPB == 0 ? e / TN : e % TK;
                const int c = c0 + cc, k = k0 + kk;
                C2 v = {0, 0};
                if (c < N && k < kend) {
                    v = OPB == 0 ? B[(int64_t)k * ldb + c] : B[(int64_t)c * ldb + k];
                    if (OPB == 2) v.y = -v.y;
                }
                rb[q] = v;
            }
        }
    };
    if (kbeg < kend) load(kbeg);
    for (int k0 = kbeg; k0 < kend; k0 += TK) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int e = t + 256 * q;
            As[OPA == 0 ? e % TK : e / TM][OPA == 0 ? e / TK : e % TM] = ra[q];
            Bs[OPB == 0 ? e / TN : e % TK][OPB == 0 ? e % TN : e / TK] = rb[q];
        }
        __syncthreads();
        if (k0 + TK < kend) load(k0 + TK);
#pragma unroll
        for (int k4 = 0; k4 < TK / 4; ++k4) {
            const int kk = 4 * k4 + fk;
            C2 av[2], bv[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) av[i] = As[kk][wm * 32 + i * 16 + fr];
#pragma unroll
            for (int j = 0; j < 2; ++j) bv[j] = Bs[kk][wn * 32 + j * 16 + fr];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    accr[i][j] = ZT<T>::mfma(av[i].x, bv[j].x, accr[i][j]);
                    accr[i][j] = ZT<T>::mfma(-av[i].y, bv[j].y, accr[i][j]);
                    acci[i][j] = ZT<T>::mfma(av[i].x, bv[j].y, acci[i][j]);
                    acci[i][j] = ZT<T>::mfma(av[i].y, bv[j].x, acci[i][j]);
                }
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int r = r0 + wm * 32 + i * 16 + ZT<T>::row(q, fk), c = c0 + wn * 32 + j * 16 + fr;
                if (r < M && c < N) {
                    int64_t at;
                    if constexpr (XC) {
                        const int64_t r1 = r / xm, r2 = r - r1 * xm, c1 = c / xv, c2 = c - c1 * xv;
                        at = ((r1 * xm + c1) * xm + r2) * xv + c2;
                    } else {
                        at = (int64_t)r * ldc + c;
                    }
                    C2 &o = C[at];
                    if (sub) {
                        o.x -= accr[i][j][q];
                        o.y -= acci[i][j][q];
                    } else {
                        o.x = accr[i][j][q];
                        o.y = acci[i][j][q];
                    }
                }
            }
}

// out[i] = (float2) in[i]
__global__ void __launch_bounds__(256) k_to_c64(const double2 *__restrict__ in, int64_t n, float2 *__restrict__ out) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        out[e] = make_float2((float)in[e].x, (float)in[e].y);
}

// out[b][j][i][k] = in[b][i][j][k] for float2 tensors (the FP32 factorised
// operator's axis exchange)
__global__ void __launch_bounds__(256) k_swap01_c64(const float2 *__restrict__ in, int64_t nb, int64_t n0, int64_t n1,
                                                    int64_t n2, float2 *__restrict__ out) {
    const int64_t per = n0 * n1 * n2, total = nb * per;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
        const int64_t bb = e / per, r = e % per;
        const int64_t k = r % n2, j = (r / n2) % n1, i = r / (n1 * n2);
        out[bb * per + (j * n0 + i) * n2 + k] = in[e];
    }
}

// out[b][j][i][k] = in[b][i][j][k] for nb tensors of shape (n0, n1, n2)
// (exchange of their first two axes), conjugated if asked.
__global__ void __launch_bounds__(256) k_swap01(const double2 *__restrict__ in, int64_t nb, int64_t n0, int64_t n1,
                                                int64_t n2, int conj, double2 *__restrict__ out) {
    const int64_t per = n0 * n1 * n2, total = nb * per;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
        const int64_t b = e / per, r = e % per;
        const int64_t k = r % n2, j = (r / n2) % n1, i = r / (n1 * n2);
        double2 v = in[e];
        if (conj) v.y = -v.y;
        out[b * per + (j * n0 + i) * n2 + k] = v;
    }
}

// Partial sums of |x|^2 (one per block) and their total in one thread.
__global__ void __launch_bounds__(256) k_sumsq(const double2 *__restrict__ x, int64_t n, double *__restrict__ part) {
    __shared__ double sh[256];
    double s = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        s += x[e].x * x[e].x + x[e].y * x[e].y;
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}
__global__ void k_sum_parts(double *__restrict__ part, int n) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += part[i];
    part[n] = s;
}

// The effective state: from T[(kA, u)][w][(kB, v)] into psi[(a, b, e)] with
// zero padding to dA2 x dB2 x dE2 (powers of two), e = (u W + w) V + v, all
// scaled by 1 / sqrt(sumsq).
// s = Re sum_i A[i] conj(C[i]) over n entries (one block), written to out[0].
__global__ void __launch_bounds__(256) k_dot_re(const double2 *__restrict__ A, const double2 *__restrict__ C,
                                                int64_t n, double *__restrict__ out) {
    __shared__ double sh[256];
    double s = 0.0;
    for (int64_t e = threadIdx.x; e < n; e += 256) s += A[e].x * C[e].x + A[e].y * C[e].y;
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = sh[0];
}

// x *= 1 / sqrt(s[0])
__global__ void __launch_bounds__(256) k_scale_rsqrt(double2 *__restrict__ x, int64_t n, const double *__restrict__ s) {
    const double f = 1.0 / sqrt(s[0]);
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        x[e].x *= f;
        x[e].y *= f;
    }
}

__global__ void __launch_bounds__(256) k_assemble(const double2 *__restrict__ T, int64_t kA, int64_t U, int64_t W,
                                                  int64_t kB, int64_t V, int64_t dB2, int64_t dE2, int64_t total,
                                                  const double *__restrict__ sumsq, double2 *__restrict__ psi) {
    const double sc = 1.0 / sqrt(*sumsq);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; o < total; o += stride) {
        const int64_t e = o % dE2, b = (o / dE2) % dB2, a = o / (dE2 * dB2);
        double2 v = make_double2(0.0, 0.0);
        if (a < kA && b < kB && e < U * W * V) {
            const int64_t vv = e % V, w = (e / V) % W, u = e / (V * W);
            v = T[((a * U + u) * W + w) * (kB * V) + b * V + vv];
            v = make_double2(v.x * sc, v.y * sc);
        }
        psi[o] = v;
    }
}

// ---------------------------------------------------------------------------
// Transfer matrices of sections (the first step of Sec. VI's lateral
// compression): T[(x, x')][y'][y] = sum_s S[x][s][y] conj(S[x'][s][y']) for a
// section S with left bond x and right bond y, built one site at a time.

// T0[(u, u')][z'][z] = X[z][u] conj(X[z'][u']) for an n x n factor X (the
// identity when X is null): the transfer matrix of no sites with X absorbed
// on the left bond.
__global__ void __launch_bounds__(256) k_transfer_start(const double2 *__restrict__ X, int64_t n,
                                                        double2 *__restrict__ T) {
    const int64_t total = n * n * n * n;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t z = e % n, zp = (e / n) % n, up = (e / (n * n)) % n, u = e / (n * n * n);
        double2 v;
        if (X) {
            const double2 a = X[z * n + u], b = X[zp * n + up];
            v = cmul(a, cconj(b));
        } else {
            v = make_double2(z == u && zp == up ? 1.0 : 0.0, 0.0);
        }
        T[e] = v;
    }
}

// s = sum_{a < x, c < y} Re T[(a, a)][c][c] (one block; 256 partial sums
// combined in a fixed order).
__global__ void __launch_bounds__(256) k_transfer_trace(const double2 *__restrict__ T, int64_t x, int64_t y,
                                                        double *__restrict__ s) {
    __shared__ double sh[256];
    double acc = 0.0;
    for (int64_t e = threadIdx.x; e < x * y; e += 256) {
        const int64_t a = e / y, c = e % y;
        acc += T[((a * x + a) * y + c) * y + c].x;
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) s[0] = sh[0];
}

// x /= s[0] where s[0] > 0 (a zero or non-finite trace leaves x as it is; the
// factorisation then reports what it finds)
__global__ void __launch_bounds__(256) k_scale_inv(double2 *__restrict__ x, int64_t n, const double *__restrict__ s) {
    const double t = s[0];
    if (!(t > 0.0) || !isfinite(t)) return;
    const double f = 1.0 / t;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        x[e].x *= f;
        x[e].y *= f;
    }
}

// out[b] = in[b] with its four axes permuted, for nb tensors one after the
// other: in[b] has shape d[0..3], out axis j is in axis perm[j] (out shape
// d[perm[0]], ..., d[perm[3]]).
struct Perm4 {
    int64_t od[4];   // out shape
    int64_t is[4];   // in stride of out axis j
    int64_t per;     // entries per tensor
};
template <typename T>
__global__ void __launch_bounds__(256) k_permute4(const T *__restrict__ in, Perm4 p, int64_t total,
                                                  T *__restrict__ out) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b = e / p.per;
        int64_t r = e - b * p.per, off = b * p.per;
#pragma unroll
        for (int j = 3; j >= 0; --j) {
            off += (r % p.od[j]) * p.is[j];
            r /= p.od[j];
        }
        out[e] = in[off];
    }
}

// out[i][j] = delta(i, j), n x n
__global__ void __launch_bounds__(256) k_identity(double2 *__restrict__ out, int64_t n) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n * n; e += (int64_t)gridDim.x * blockDim.x)
        out[e] = make_double2(e / n == e % n ? 1.0 : 0.0, 0.0);
}

unsigned blocks_for(int64_t n) {
    int64_t g = (n + 255) / 256;
    if (g < 1) g = 1;
    if (g > 65535 * 8) g = 65535 * 8;
    return (unsigned)g;
}

}  // namespace

// Left: E_new[y][y'] = sum_{x, x', s} E[x][x'] M[x][s][y] conj(M[x'][s][y'])
// as G[x][(s, y)] = sum_x' E[x'][x] M[x'][(s, y)], H = M^dagger G over (x, s),
// E_new = H^T.  Right: E_new[x][x'] = sum_{y, y', s} M[x][s][y]
// conj(M[x'][s][y']) E[y][y'] as G = M E over y, E_new = G conj(M)^T over
// (s, y').  Two complex products of chi^3 p multiply-adds each.
hipError_t launch_transfer(int left, const double2 *E, const double2 *M, int cx, int p, int cy, double2 *Enew,
                           double2 *tmp, hipStream_t st) {
    const int nout = left ? cy : cx;
    const int64_t pcy = (int64_t)p * cy;
    hipError_t e;
    if (left) {
        double2 *G = tmp, *H = tmp + (int64_t)cx * pcy;
        if ((e = launch_zgemm(1, 0, E, M, G, cx, (int)pcy, cx, cx, pcy, pcy, 1, 0, 0, 0, st)) != hipSuccess) return e;
        if ((e = launch_zgemm(2, 0, M, G, H, cy, cy, cx * p, cy, cy, cy, 1, 0, 0, 0, st)) != hipSuccess) return e;
        if ((e = launch_swap01(H, 1, cy, cy, 1, 0, Enew, st)) != hipSuccess) return e;
    } else {
        double2 *G = tmp;
        if ((e = launch_zgemm(0, 0, M, E, G, cx * p, cy, cy, cy, cy, cy, 1, 0, 0, 0, st)) != hipSuccess) return e;
        if ((e = launch_zgemm(0, 2, G, M, Enew, cx, cx, (int)pcy, pcy, pcy, cx, 1, 0, 0, 0, st)) != hipSuccess)
            return e;
    }
    hipLaunchKernelGGL(k_scale_by_trace, dim3(1), dim3(256), 0, st, Enew, nout);
    return hipGetLastError();
}

hipError_t launch_cholesky(double2 *A, int n, int *fail, double *dmax, hipStream_t st) {
    if (n < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_chol_init, dim3(1), dim3(256), 0, st, A, n, dmax);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    for (int j0 = 0; j0 < n; j0 += CNB) {
        const int w = n - j0 < CNB ? n - j0 : CNB, rest = n - j0 - w;
        hipLaunchKernelGGL(k_chol_panel, dim3(1), dim3(256), 0, st, A, n, j0, dmax, fail);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if (rest == 0) break;
        hipLaunchKernelGGL(k_chol_trsm, dim3((rest + 255) / 256), dim3(256), 0, st, A, n, j0);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        // A22 -= L21 L21^dagger (the full square; its upper part is zeroed last)
        const double2 *L21 = A + (int64_t)(j0 + w) * n + j0;
        if ((e = launch_zgemm(0, 2, L21, L21, A + (int64_t)(j0 + w) * n + j0 + w, rest, rest, w, n, n, n, 1, 0, 0, 0,
                              st, 1)) != hipSuccess)
            return e;
    }
    hipLaunchKernelGGL(k_zero_upper, dim3(blocks_for((int64_t)n * n)), dim3(256), 0, st, A, n);
    return hipGetLastError();
}

template <typename T>
hipError_t zgemm_t(int opa, int opb, const typename ZT<T>::C2 *A, const typename ZT<T>::C2 *B, typename ZT<T>::C2 *C,
                   int M, int N, int K, int64_t lda, int64_t ldb, int64_t ldc, int batch, int64_t sa, int64_t sb,
                   int64_t sc, hipStream_t st, int sub, int ks, int64_t csk) {
    if (batch < 1 || ks < 1 || (int64_t)batch * ks > 65535 || (sub && ks > 1)) return hipErrorInvalidValue;
    // rows in chunks of 65535 tiles (the grid's y limit)
    constexpr int64_t RCH = 65535 * 64;
    for (int64_t r0 = 0; r0 < M; r0 += RCH) {
        const int m = (int)(M - r0 < RCH ? M - r0 : RCH);
        const typename ZT<T>::C2 *Ac = opa == 0 ? A + r0 * lda : A + r0;
        typename ZT<T>::C2 *Cc = C + r0 * ldc;
        dim3 grid((unsigned)((N + 63) / 64), (unsigned)((m + 63) / 64), (unsigned)(batch * ks)), block(256);
#define TNSLQ_ZG(OA, OB)                                                                                       \
    hipLaunchKernelGGL((k_zgemm<OA, OB, T>), grid, block, 0, st, Ac, B, Cc, m, N, K, lda, ldb, ldc, sa, sb, sc, sub, \
                       ks, csk)
        if (opa == 0 && opb == 0) TNSLQ_ZG(0, 0);
        else if (opa == 1 && opb == 0) TNSLQ_ZG(1, 0);
        else if (opa == 2 && opb == 0) TNSLQ_ZG(2, 0);
        else if (opa == 0 && opb == 2) TNSLQ_ZG(0, 2);
        else return hipErrorInvalidValue;
#undef TNSLQ_ZG
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_zgemm(int opa, int opb, const double2 *A, const double2 *B, double2 *C, int M, int N, int K,
                        int64_t lda, int64_t ldb, int64_t ldc, int batch, int64_t sa, int64_t sb, int64_t sc,
                        hipStream_t st, int sub, int ks, int64_t csk) {
    return zgemm_t<double>(opa, opb, A, B, C, M, N, K, lda, ldb, ldc, batch, sa, sb, sc, st, sub, ks, csk);
}

template <typename T>
static hipError_t zgemm_xc_t(const typename ZT<T>::C2 *A, const typename ZT<T>::C2 *B, typename ZT<T>::C2 *C, int M,
                             int N, int K, int64_t lda, int64_t ldb, int batch, int64_t sa, int64_t sb, int64_t sc,
                             int64_t xm, int64_t xv, hipStream_t st) {
    // one launch (rows within the grid's y limit), whole row and column groups
    if (batch < 1 || batch > 65535 || (int64_t)M > 65535 * 64 || xm < 1 || xv < 1 || M % xm || N % xv)
        return hipErrorInvalidValue;
    dim3 grid((unsigned)((N + 63) / 64), (unsigned)((M + 63) / 64), (unsigned)batch), block(256);
    hipLaunchKernelGGL((k_zgemm<0, 0, T, true>), grid, block, 0, st, A, B, C, M, N, K, lda, ldb, (int64_t)0, sa, sb,
                       sc, 0, 1, (int64_t)0, xm, xv);
    return hipGetLastError();
}

hipError_t launch_zgemm_xc(const double2 *A, const double2 *B, double2 *C, int M, int N, int K, int64_t lda,
                           int64_t ldb, int batch, int64_t sa, int64_t sb, int64_t sc, int64_t xm, int64_t xv,
                           hipStream_t st) {
    return zgemm_xc_t<double>(A, B, C, M, N, K, lda, ldb, batch, sa, sb, sc, xm, xv, st);
}

hipError_t launch_zgemm_xc(const float2 *A, const float2 *B, float2 *C, int M, int N, int K, int64_t lda,
                           int64_t ldb, int batch, int64_t sa, int64_t sb, int64_t sc, int64_t xm, int64_t xv,
                           hipStream_t st) {
    return zgemm_xc_t<float>(A, B, C, M, N, K, lda, ldb, batch, sa, sb, sc, xm, xv, st);
}

hipError_t launch_zgemm(int opa, int opb, const float2 *A, const float2 *B, float2 *C, int M, int N, int K,
                        int64_t lda, int64_t ldb, int64_t ldc, int batch, int64_t sa, int64_t sb, int64_t sc,
                        hipStream_t st, int sub, int ks, int64_t csk) {
    return zgemm_t<float>(opa, opb, A, B, C, M, N, K, lda, ldb, ldc, batch, sa, sb, sc, st, sub, ks, csk);
}

hipError_t launch_to_c64(const double2 *in, int64_t n, float2 *out, hipStream_t st) {
    hipLaunchKernelGGL(k_to_c64, dim3(blocks_for(n)), dim3(256), 0, st, in, n, out);
    return hipGetLastError();
}

hipError_t launch_swap01(const float2 *in, int64_t nb, int64_t n0, int64_t n1, int64_t n2, float2 *out,
                         hipStream_t st) {
    hipLaunchKernelGGL(k_swap01_c64, dim3(blocks_for(nb * n0 * n1 * n2)), dim3(256), 0, st, in, nb, n0, n1, n2, out);
    return hipGetLastError();
}

hipError_t launch_swap01(const double2 *in, int64_t nb, int64_t n0, int64_t n1, int64_t n2, int conj, double2 *out,
                         hipStream_t st) {
    hipLaunchKernelGGL(k_swap01, dim3(blocks_for(nb * n0 * n1 * n2)), dim3(256), 0, st, in, nb, n0, n1, n2, conj, out);
    return hipGetLastError();
}

hipError_t launch_sumsq(const double2 *x, int64_t n, double *part, hipStream_t st) {
    hipLaunchKernelGGL(k_sumsq, dim3(256), dim3(256), 0, st, x, n, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(1), 0, st, part, 256);
    return hipGetLastError();
}

hipError_t launch_normalise_factor(const double2 *Ahat, const double2 *C, int64_t mm, double *nrm, double2 *P,
                                   int64_t np, hipStream_t st) {
    hipLaunchKernelGGL(k_dot_re, dim3(1), dim3(256), 0, st, Ahat, C, mm, nrm);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_scale_rsqrt, dim3(blocks_for(np)), dim3(256), 0, st, P, np, nrm);
    return hipGetLastError();
}

hipError_t launch_assemble(const double2 *T, int64_t kA, int64_t U, int64_t W, int64_t kB, int64_t V, int64_t dA2,
                           int64_t dB2, int64_t dE2, const double *sumsq, double2 *psi, hipStream_t st) {
    const int64_t total = dA2 * dB2 * dE2;
    hipLaunchKernelGGL(k_assemble, dim3(blocks_for(total)), dim3(256), 0, st, T, kA, U, W, kB, V, dB2, dE2, total, sumsq,
                       psi);
    return hipGetLastError();
}

// Batched C[b] = op(A) B[b] in chunks of at most 65535 batch entries (the
// grid's z limit).
static hipError_t zgemm_batches(int opa, const double2 *A, const double2 *B, double2 *C, int M, int N, int K,
                                int64_t lda, int64_t ldb, int64_t ldc, int64_t batch, int64_t sb, int64_t sc,
                                hipStream_t st) {
    for (int64_t b0 = 0; b0 < batch; b0 += 65535) {
        const int nb = (int)(batch - b0 < 65535 ? batch - b0 : 65535);
        hipError_t e = launch_zgemm(opa, 0, A, B + b0 * sb, C + b0 * sc, M, N, K, lda, ldb, ldc, nb, 0, sb, sc, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

static hipError_t scale_by_transfer_trace(double2 *T, int64_t x, int64_t y, double *s, hipStream_t st) {
    hipLaunchKernelGGL(k_transfer_trace, dim3(1), dim3(256), 0, st, T, x, y, s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t n = x * x * y * y;
    hipLaunchKernelGGL(k_scale_inv, dim3(blocks_for(n)), dim3(256), 0, st, T, n, s);
    return hipGetLastError();
}

hipError_t launch_transfer_start(const double2 *X, int64_t n, double2 *T, double *s, hipStream_t st) {
    const int64_t total = n * n * n * n;
    hipLaunchKernelGGL(k_transfer_start, dim3(blocks_for(total)), dim3(256), 0, st, X, n, T);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return scale_by_transfer_trace(T, n, n, s, st);
}

// One site M[z][s][y] (cz x p x cy) onto T[(x, x')][z'][z]:
//   A[(r, z')][(s, y)] = sum_z T[(r, z')][z] M[z][(s, y)]          (one product)
//   Tnew[r][y'][y]     = sum_(z', s) conj(M[(z', s)][y']) A[r][(z', s)][y]  (x^2 products)
// then Tnew divided by its trace.  x^2 p cz cy (cz + cy) complex multiply-adds.
hipError_t launch_transfer_step(const double2 *T, const double2 *M, int64_t x, int64_t cz, int64_t p, int64_t cy,
                                double2 *Tnew, double2 *A, double *s, hipStream_t st) {
    const int64_t r = x * x, pcy = p * cy;
    hipError_t e = launch_zgemm(0, 0, T, M, A, (int)(r * cz), (int)pcy, (int)cz, cz, pcy, pcy, 1, 0, 0, 0, st);
    if (e != hipSuccess) return e;
    if ((e = zgemm_batches(2, M, A, Tnew, (int)cy, (int)cy, (int)(cz * p), cy, cy, cy, r, cz * pcy, cy * cy, st)) !=
        hipSuccess)
        return e;
    return scale_by_transfer_trace(Tnew, x, cy, s, st);
}

// T -> T' of the section S Y (Y: cy x cv): H[(r, y')][v] = sum_y T[(r, y')][y]
// Y[y][v], T'[r][v'][v] = sum_y' conj(Y[y'][v']) H[r][y'][v].
hipError_t launch_transfer_absorb_right(const double2 *T, const double2 *Y, int64_t x, int64_t cy, int64_t cv,
                                        double2 *Tnew, double2 *H, double *s, hipStream_t st) {
    const int64_t r = x * x;
    hipError_t e = launch_zgemm(0, 0, T, Y, H, (int)(r * cy), (int)cv, (int)cy, cy, cv, cv, 1, 0, 0, 0, st);
    if (e != hipSuccess) return e;
    if ((e = zgemm_batches(2, Y, H, Tnew, (int)cv, (int)cv, (int)cy, cv, cv, cv, r, cy * cv, cv * cv, st)) !=
        hipSuccess)
        return e;
    return scale_by_transfer_trace(Tnew, x, cv, s, st);
}

template <typename T>
static hipError_t permute4_t(const T *in, const int64_t d[4], const int perm[4], T *out, hipStream_t st, int64_t nb) {
    Perm4 p;
    int64_t stride[4];
    stride[3] = 1;
    for (int j = 2; j >= 0; --j) stride[j] = stride[j + 1] * d[j + 1];
    int seen = 0;
    for (int j = 0; j < 4; ++j) {
        if (perm[j] < 0 || perm[j] > 3 || (seen >> perm[j]) & 1) return hipErrorInvalidValue;
        seen |= 1 << perm[j];
        p.od[j] = d[perm[j]];
        p.is[j] = stride[perm[j]];
    }
    p.per = d[0] * d[1] * d[2] * d[3];
    const int64_t total = nb * p.per;
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL(k_permute4<T>, dim3(blocks_for(total)), dim3(256), 0, st, in, p, total, out);
    return hipGetLastError();
}

hipError_t launch_permute4(const double2 *in, const int64_t d[4], const int perm[4], double2 *out, hipStream_t st,
                           int64_t nb) {
    return permute4_t(in, d, perm, out, st, nb);
}

hipError_t launch_permute4(const float2 *in, const int64_t d[4], const int perm[4], float2 *out, hipStream_t st,
                           int64_t nb) {
    return permute4_t(in, d, perm, out, st, nb);
}

hipError_t launch_trace_pairs(const double2 *T, int64_t x, int64_t y, double *s, hipStream_t st) {
    hipLaunchKernelGGL(k_transfer_trace, dim3(1), dim3(256), 0, st, T, x, y, s);
    return hipGetLastError();
}

hipError_t launch_scale_rsqrt(double2 *x, int64_t n, const double *s, hipStream_t st) {
    hipLaunchKernelGGL(k_scale_rsqrt, dim3(blocks_for(n)), dim3(256), 0, st, x, n, s);
    return hipGetLastError();
}

hipError_t launch_identity(double2 *out, int64_t n, hipStream_t st) {
    hipLaunchKernelGGL(k_identity, dim3(blocks_for(n * n)), dim3(256), 0, st, out, n);
    return hipGetLastError();
}

}  // namespace tnslq
