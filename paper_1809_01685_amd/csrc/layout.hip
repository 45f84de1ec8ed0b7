// Operand preparation: regrouping psi into the two contraction layouts
// (Sec. IV: grouping indices turns the network into matrix products; Sec. V:
// psi_{1..L} -> psi_{abc}), the Hutchinson probe block (Sec. III,
// Algorithm 1), and the conversions between caller vectors and the
// contraction operands.
#include <algorithm>

#include "tnslq_internal.h"

namespace tnslq {
namespace {

// ---------------------------------------------------------------- psi
template <int DTYPE>
__device__ inline double2 load_psi(const void *psi, int64_t i) {
    if constexpr (DTYPE == TNSLQ_C128) {
        return ((const double2 *)psi)[i];
    } else {
        float2 v = ((const float2 *)psi)[i];
        return make_double2(v.x, v.y);
    }
}

// Brick operand of R x Kr entries from psi: entry (r, l) = psi[in(r Kr + l)]
// (conjugated if asked), where bit t of the regrouped index is bit map[t] of
// in, and zeros in the padding.  Threads step over the plane-0 entries of the
// bricks in memory order, so consecutive threads write consecutive elements of
// every plane.
template <int PREC, int DTYPE>
__global__ void __launch_bounds__(256) k_permute(const void *__restrict__ psi, void *__restrict__ out, int64_t R,
                                                 int64_t Kr, int64_t nst, PermDesc pd, int conj) {
    constexpr int EPR = brick_epr(PREC), EPU = EPR / 4, NPL = planes_of(PREC);
    constexpr int64_t PER_BRICK = (int64_t)BRICK_ROWS * EPR;
    const int64_t total = brick_rows(R) * nst * EPR;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < total; x += stride) {
        const int64_t b = x / PER_BRICK, w = x % PER_BRICK;
        const int64_t rr = w / EPR, pos = w % EPR;
        // stored unit pos / EPU holds logical unit (pos / EPU) ^ swizzle(rr)
        const int64_t ll = (((pos / EPU) ^ brick_swizzle(rr)) * EPU) + pos % EPU;
        const int64_t r = (b / nst) * BRICK_ROWS + rr, l = (b % nst) * EPR + ll;
        double2 v = make_double2(0.0, 0.0);
        if (r < R && l < Kr) {
            const int64_t o = r * Kr + l;
            int64_t in = 0;
            for (int t = 0; t < pd.L; ++t) in |= ((o >> t) & 1) << pd.map[t];
            v = load_psi<DTYPE>(psi, in);
            if (conj) v.y = -v.y;
        }
        store_planes<PREC>(out, brick_ps(PREC), (b * NPL * BRICK_ROWS + rr) * EPR + pos, v.x, v.y);
    }
}

// psi index of the digits of v in group g (most significant site first).
__device__ inline int64_t mixed_offset(const MixedDesc &md, int g, int64_t v) {
    int64_t in = 0;
    for (int i = md.n[g] - 1; i >= 0; --i) {
        const int64_t q = v / md.dim[g][i];
        in += (v - q * md.dim[g][i]) * md.stride[g][i];
        v = q;
    }
    return in;
}

// P[(a, b)][c] = psi at A's digits of a, B's of b and E's of c, as a brick
// operand of d_A d_B rows and d_E reduction terms (conjugated if asked), zeros
// in the padding; threads step over the bricks in memory order as in
// k_permute.
template <int PREC, int DTYPE>
__global__ void __launch_bounds__(256) k_permute_mixed(const void *__restrict__ psi, void *__restrict__ out,
                                                       MixedDesc md, int64_t nst, int conj) {
    constexpr int EPR = brick_epr(PREC), EPU = EPR / 4, NPL = planes_of(PREC);
    constexpr int64_t PER_BRICK = (int64_t)BRICK_ROWS * EPR;
    const int64_t R = md.d[0] * md.d[1], Kr = md.d[2];
    const int64_t total = brick_rows(R) * nst * EPR;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < total; x += stride) {
        const int64_t b = x / PER_BRICK, w = x % PER_BRICK;
        const int64_t rr = w / EPR, pos = w % EPR;
        const int64_t ll = (((pos / EPU) ^ brick_swizzle(rr)) * EPU) + pos % EPU;
        const int64_t r = (b / nst) * BRICK_ROWS + rr, l = (b % nst) * EPR + ll;
        double2 v = make_double2(0.0, 0.0);
        if (r < R && l < Kr) {
            const int64_t in = mixed_offset(md, 0, r / md.d[1]) + mixed_offset(md, 1, r % md.d[1]) +
                               mixed_offset(md, 2, l);
            v = load_psi<DTYPE>(psi, in);
            if (conj) v.y = -v.y;
        }
        store_planes<PREC>(out, brick_ps(PREC), (b * NPL * BRICK_ROWS + rr) * EPR + pos, v.x, v.y);
    }
}

// ---------------------------------------------------------------- probes
__device__ inline uint64_t splitmix64(uint64_t seed, uint64_t n) {
    // n-th output of SplitMix64 seeded with `seed` (state advances by the
    // golden gamma before each output).
    uint64_t z = seed + (n + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Probe k's value at layout position (a, b).  Without the role swap the flat
// index is a * dB + b; with it, layout (a, b) is the caller's (b, a) and the
// value is conjugated (the operator on the swapped layout is the complex
// conjugate of rho^{T_B}, so the conjugated probe reproduces the same Krylov
// coefficients).
__device__ inline double2 probe_value(uint64_t seed, uint64_t offset, int k, int64_t a, int64_t b,
                                      int64_t dA, int64_t dB, int swapped) {
    const int64_t n = dA * dB;
    const int64_t i = swapped ? (b * dA + a) : (a * dB + b);
    const uint64_t r = splitmix64(seed, (offset + (uint64_t)k) * (uint64_t)n + (uint64_t)i) >> 62;
    double re = (r == 0) ? 1.0 : (r == 2 ? -1.0 : 0.0);
    double im = (r == 1) ? 1.0 : (r == 3 ? -1.0 : 0.0);
    if (swapped) im = -im;
    return make_double2(re, im);
}

// q_1 = phi / beta_1 with beta_1 = ||phi|| = sqrt(d_A d_B) (unit-modulus
// entries), in [k][a][b] order, and its transposed low-precision copy Xt.
template <int PREC>
__global__ void __launch_bounds__(256) k_probe_init(uint64_t seed, uint64_t offset, int swapped,
                                                    int64_t dA, int64_t dB, double2 *__restrict__ q,
                                                    void *__restrict__ Xt, int64_t xt_nst,
                                                    double *__restrict__ beta, int m) {
    const int k = blockIdx.y;
    const int64_t n = dA * dB;
    const double b1 = sqrt((double)n);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) {
        // q in [a][b] order, b fastest
        const int64_t a = e / dB, b = e % dB;
        double2 v = probe_value(seed, offset, k, a, b, dA, dB, swapped);
        q[(int64_t)k * n + e] = make_double2(v.x / b1, v.y / b1);
        // Xt row (k, b'), reduction index a' (when the caller contracts through Xt)
        if (Xt) {
            const int64_t b2 = e / dA, a2 = e % dA;
            double2 u = probe_value(seed, offset, k, a2, b2, dA, dB, swapped);
            store_planes<PREC>(Xt, brick_ps(PREC), brick_index(PREC, xt_nst, (int64_t)k * dB + b2, a2), u.x / b1,
                               u.y / b1);
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) beta[(int64_t)k * (m + 1)] = b1;
}

// Plain probe block for the caller (complex128, caller's index order).
__global__ void k_probes(uint64_t seed, uint64_t offset, int64_t d, double2 *__restrict__ X) {
    const int k = blockIdx.y;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < d; i += stride)
        X[(int64_t)k * d + i] = probe_value(seed, offset, k, i / d, i % d, 1, d, 0);
}

// Caller vectors X[k][a_o][b_o] -> contraction operand Xt, row (k, b),
// reduction index a, in layout roles (conjugated and index-swapped when the
// roles are swapped).
template <int PREC>
__global__ void __launch_bounds__(256) k_load_vectors(const double2 *__restrict__ X, int64_t dA,
                                                      int64_t dB, int swapped, void *__restrict__ Xt,
                                                      int64_t xt_nst) {
    const int k = blockIdx.y;
    const int64_t n = dA * dB;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) {
        const int64_t b = e / dA, a = e % dA;   // Xt position [b][a]
        double2 v;
        if (swapped) {
            v = X[(int64_t)k * n + b * dA + a];  // caller (a_o, b_o) = (b, a)
            v.y = -v.y;
        } else {
            v = X[(int64_t)k * n + a * dB + b];
        }
        store_planes<PREC>(Xt, brick_ps(PREC), brick_index(PREC, xt_nst, (int64_t)k * dB + b, a), v.x, v.y);
    }
}

// Caller vectors X[k][a_o][b_o] -> FP64 vectors in layout order, Xs[k][a dB + b]
// (conjugated and index-swapped when the roles are swapped), for the
// streaming form of the contractions.
__global__ void __launch_bounds__(256) k_load_vectors_plain(const double2 *__restrict__ X, int64_t dA, int64_t dB,
                                                            int swapped, double2 *__restrict__ Xs) {
    const int k = blockIdx.y;
    const int64_t n = dA * dB;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) {
        const int64_t a = e / dB, b = e % dB;
        double2 v;
        if (swapped) {
            v = X[(int64_t)k * n + b * dA + a];
            v.y = -v.y;
        } else {
            v = X[(int64_t)k * n + e];
        }
        Xs[(int64_t)k * n + e] = v;
    }
}

// Y = sum over split-K partials, written in the caller's index order.
template <typename AccT>
__global__ void __launch_bounds__(256) k_reduce_partials(const AccT *__restrict__ part, int S,
                                                         int64_t split_stride, int64_t dA, int64_t dB,
                                                         int swapped, double2 *__restrict__ Y) {
    const int k = blockIdx.y;
    const int64_t n = dA * dB;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) {
        // e indexes the caller's order
        int64_t src;
        if (swapped) {
            // caller (a_o, b_o) = layout (b, a): e = a_o * dB_o + b_o, dB_o = dA
            const int64_t ao = e / dA, bo = e % dA;
            src = bo * dB + ao;
        } else {
            src = e;
        }
        double re = 0.0, im = 0.0;
        for (int s = 0; s < S; ++s) {
            AccT v = part[s * split_stride + (int64_t)k * n + src];
            re += (double)v.x;
            im += (double)v.y;
        }
        Y[(int64_t)k * n + e] = make_double2(re, swapped ? -im : im);
    }
}

// The first contraction split along its reduction: the S partial sums of
// Ups[k][(b, c)][b'] (accumulator type, at s * split + k * M dB + (b dE + c) dB
// + b' with M = dB dE) added in FP64 and stored into the Ups brick operand,
// row k dB + b, reduction index c dB + b'.
template <int PREC, typename AccT>
__global__ void __launch_bounds__(256) k_partials_to_bricks(const AccT *__restrict__ part, int S, int64_t split,
                                                            int64_t n, int nB, int nE, void *__restrict__ ups,
                                                            int64_t ups_nst) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t dB = int64_t(1) << nB, dE = int64_t(1) << nE;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) {
        double re = 0.0, im = 0.0;
        for (int s = 0; s < S; ++s) {
            const AccT v = part[s * split + e];
            re += (double)v.x;
            im += (double)v.y;
        }
        const int64_t bp = e & (dB - 1), i = (e >> nB) % (dB * dE), k = (e >> nB) / (dB * dE);
        const int64_t b = i >> nE, c = i & (dE - 1);
        store_planes<PREC>(ups, brick_ps(PREC), brick_index(PREC, ups_nst, k * dB + b, (c << nB) + bp), re, im);
    }
}

// ---------------------------------------------------------- explicit operator
// Intermediary (iii) of Sec. V from the dense product C = rho_AB (row-major
// n x n, accumulator type AccT): exchanging B's bra and ket indices,
//   rho^{T_B}[(a, b)][(a', b')] = C[(a, b')][(a', b)],
// written as an n x n brick operand (rows (a, b), reduction index (a', b')),
// zeros in the reduction padding.  Threads step over the plane-0 entries of
// the bricks in memory order, as in k_permute.
template <int PREC, typename AccT>
__global__ void __launch_bounds__(256) k_pt_bricks(const AccT *__restrict__ C, int64_t n, int64_t dB,
                                                   void *__restrict__ rho, int64_t nst) {
    constexpr int EPR = brick_epr(PREC), EPU = EPR / 4, NPL = planes_of(PREC);
    constexpr int64_t PER_BRICK = (int64_t)BRICK_ROWS * EPR;
    const int64_t total = brick_rows(n) * nst * EPR;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < total; x += stride) {
        const int64_t b = x / PER_BRICK, w = x % PER_BRICK;
        const int64_t rr = w / EPR, pos = w % EPR;
        const int64_t ll = (((pos / EPU) ^ brick_swizzle(rr)) * EPU) + pos % EPU;
        const int64_t r = (b / nst) * BRICK_ROWS + rr, l = (b % nst) * EPR + ll;
        double re = 0.0, im = 0.0;
        if (r < n && l < n) {
            const int64_t rb = r % dB, lb = l % dB;
            const AccT v = C[(r - rb + lb) * n + (l - lb + rb)];
            re = (double)v.x;
            im = (double)v.y;
        }
        store_planes<PREC>(rho, brick_ps(PREC), (b * NPL * BRICK_ROWS + rr) * EPR + pos, re, im);
    }
}

// The same as a dense complex128 matrix, one thread per output element.
__global__ void __launch_bounds__(256) k_pt_dense(const double2 *__restrict__ C, int64_t n, int64_t dB,
                                                  double2 *__restrict__ out) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n * n; x += stride) {
        const int64_t r = x / n, l = x % n, rb = r % dB, lb = l % dB;
        out[x] = C[(r - rb + lb) * n + (l - lb + rb)];
    }
}

inline unsigned grid_for(int64_t n, int64_t per_block, unsigned cap) {
    int64_t g = (n + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (unsigned)g;
}

// Zero n16 16-byte units and then `tail` single bytes (a fill kernel rather
// than a memset node, so that work a caller captures into a HIP graph replays
// correctly).
__global__ void k_zero(uint4 *__restrict__ p, int64_t n16, unsigned char *__restrict__ tailp, int tail) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = i; k < n16; k += stride) p[k] = make_uint4(0u, 0u, 0u, 0u);
    if (i < tail) tailp[i] = 0;
}

// ||psi||^2 and the number of non-finite amplitudes: per-block partial sums
// (grid-stride, FP64), then one thread adds the blocks in order.
template <typename T>
__global__ void __launch_bounds__(256) k_state_partial(const T *__restrict__ psi, int64_t D,
                                                       double *__restrict__ part) {
    __shared__ double sh[2][256];
    double s = 0.0, bad = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < D; i += stride) {
        const double re = psi[i].x, im = psi[i].y;
        if (isfinite(re) && isfinite(im))
            s += re * re + im * im;
        else
            bad += 1.0;
    }
    sh[0][threadIdx.x] = s;
    sh[1][threadIdx.x] = bad;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            sh[0][threadIdx.x] += sh[0][threadIdx.x + o];
            sh[1][threadIdx.x] += sh[1][threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = sh[0][0];
        part[2 * blockIdx.x + 1] = sh[1][0];
    }
}

__global__ void k_state_sum(const double *__restrict__ part, int nb, double *__restrict__ out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double s = 0.0, bad = 0.0;
    for (int b = 0; b < nb; ++b) {
        s += part[2 * b];
        bad += part[2 * b + 1];
    }
    out[0] = s;
    out[1] = bad;
}

}  // namespace

hipError_t launch_state_check(int dtype, const void *psi, int64_t D, double *scratch, hipStream_t st) {
    const int nb = (int)std::max<int64_t>(1, std::min<int64_t>(STATE_CHECK_BLOCKS, (D + 4095) / 4096));
    double *out = scratch + 2 * STATE_CHECK_BLOCKS;
    if (dtype == TNSLQ_C128)
        hipLaunchKernelGGL(k_state_partial<double2>, dim3(nb), dim3(256), 0, st, (const double2 *)psi, D, scratch);
    else
        hipLaunchKernelGGL(k_state_partial<float2>, dim3(nb), dim3(256), 0, st, (const float2 *)psi, D, scratch);
    hipLaunchKernelGGL(k_state_sum, dim3(1), dim3(64), 0, st, (const double *)scratch, nb, out);
    return hipGetLastError();
}

hipError_t launch_zero(void *p, size_t bytes, hipStream_t st) {
    if (bytes == 0) return hipSuccess;
    if (!p || (uintptr_t)p % 16) return hipErrorInvalidValue;
    const int64_t n16 = (int64_t)(bytes / 16);
    const int tail = (int)(bytes % 16);
    const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>(4096, (n16 + 255) / 256));
    hipLaunchKernelGGL(k_zero, dim3((unsigned)blocks), dim3(256), 0, st, (uint4 *)p, n16,
                       (unsigned char *)p + n16 * 16, tail);
    return hipGetLastError();
}

hipError_t launch_permute(int prec, int dtype, const void *psi, void *out, int64_t R, int64_t Kr,
                          const PermDesc &pd, int conj, hipStream_t st) {
    const int64_t nst = brick_stages(prec, Kr);
    dim3 grid(grid_for(brick_rows(R) * nst * brick_epr(prec), 256 * 4, 65535 * 8)), block(256);
#define TNSLQ_PERM(P, T) \
    hipLaunchKernelGGL((k_permute<P, T>), grid, block, 0, st, psi, out, R, Kr, nst, pd, conj)
    if (dtype == TNSLQ_C128) {
        switch (prec) {
            case TNSLQ_FP64: TNSLQ_PERM(TNSLQ_FP64, TNSLQ_C128); break;
            case TNSLQ_FP32: TNSLQ_PERM(TNSLQ_FP32, TNSLQ_C128); break;
            case TNSLQ_BF16X3: TNSLQ_PERM(TNSLQ_BF16X3, TNSLQ_C128); break;
            default: TNSLQ_PERM(TNSLQ_BF16X6, TNSLQ_C128); break;
        }
    } else {
        switch (prec) {
            case TNSLQ_FP64: TNSLQ_PERM(TNSLQ_FP64, TNSLQ_C64); break;
            case TNSLQ_FP32: TNSLQ_PERM(TNSLQ_FP32, TNSLQ_C64); break;
            case TNSLQ_BF16X3: TNSLQ_PERM(TNSLQ_BF16X3, TNSLQ_C64); break;
            default: TNSLQ_PERM(TNSLQ_BF16X6, TNSLQ_C64); break;
        }
    }
#undef TNSLQ_PERM
    return hipGetLastError();
}

hipError_t launch_probe_init(int prec, const LzDims &z, uint64_t seed, uint64_t offset, int swapped,
                             double2 *q, void *Xt, int64_t xt_nst, double *alpha, double *beta,
                             hipStream_t st) {
    (void)alpha;
    dim3 grid(grid_for(z.n, 256 * 8, 4096), z.K), block(256);
#define TNSLQ_PI(P) \
    hipLaunchKernelGGL((k_probe_init<P>), grid, block, 0, st, seed, offset, swapped, z.dA, z.dB, q, Xt, xt_nst, beta, z.m)
    switch (prec) {
        case TNSLQ_FP64: TNSLQ_PI(TNSLQ_FP64); break;
        case TNSLQ_FP32: TNSLQ_PI(TNSLQ_FP32); break;
        case TNSLQ_BF16X3: TNSLQ_PI(TNSLQ_BF16X3); break;
        default: TNSLQ_PI(TNSLQ_BF16X6); break;
    }
#undef TNSLQ_PI
    return hipGetLastError();
}

hipError_t launch_probes_plain(uint64_t seed, uint64_t offset, int K, int64_t d, double2 *X,
                               hipStream_t st) {
    dim3 grid(grid_for(d, 256 * 8, 4096), K), block(256);
    hipLaunchKernelGGL(k_probes, grid, block, 0, st, seed, offset, d, X);
    return hipGetLastError();
}

hipError_t launch_load_vectors(int prec, const double2 *X, int64_t dA, int64_t dB, int K, int swapped,
                               void *Xt, int64_t xt_nst, hipStream_t st) {
    dim3 grid(grid_for(dA * dB, 256 * 8, 4096), K), block(256);
#define TNSLQ_LV(P) hipLaunchKernelGGL((k_load_vectors<P>), grid, block, 0, st, X, dA, dB, swapped, Xt, xt_nst)
    switch (prec) {
        case TNSLQ_FP64: TNSLQ_LV(TNSLQ_FP64); break;
        case TNSLQ_FP32: TNSLQ_LV(TNSLQ_FP32); break;
        case TNSLQ_BF16X3: TNSLQ_LV(TNSLQ_BF16X3); break;
        default: TNSLQ_LV(TNSLQ_BF16X6); break;
    }
#undef TNSLQ_LV
    return hipGetLastError();
}

hipError_t launch_reduce_partials(int accfp64, const void *part, int S, int64_t split_stride, int64_t dA,
                                  int64_t dB, int K, int swapped, double2 *Y, hipStream_t st) {
    dim3 grid(grid_for(dA * dB, 256 * 8, 4096), K), block(256);
    if (accfp64)
        hipLaunchKernelGGL((k_reduce_partials<double2>), grid, block, 0, st, (const double2 *)part, S,
                           split_stride, dA, dB, swapped, Y);
    else
        hipLaunchKernelGGL((k_reduce_partials<float2>), grid, block, 0, st, (const float2 *)part, S,
                           split_stride, dA, dB, swapped, Y);
    return hipGetLastError();
}

hipError_t launch_partials_to_bricks(int prec, const void *part, int S, int64_t split, int64_t n, int nB, int nE,
                                     void *ups, int64_t ups_nst, hipStream_t st) {
    dim3 grid(grid_for(n, 256 * 4, 65535 * 4)), block(256);
#define TNSLQ_P2B(P, A) \
    hipLaunchKernelGGL((k_partials_to_bricks<P, A>), grid, block, 0, st, (const A *)part, S, split, n, nB, nE, ups, ups_nst)
    switch (prec) {
        case TNSLQ_FP64: TNSLQ_P2B(TNSLQ_FP64, double2); break;
        case TNSLQ_FP32: TNSLQ_P2B(TNSLQ_FP32, float2); break;
        case TNSLQ_BF16X3: TNSLQ_P2B(TNSLQ_BF16X3, float2); break;
        default: TNSLQ_P2B(TNSLQ_BF16X6, float2); break;
    }
#undef TNSLQ_P2B
    return hipGetLastError();
}

hipError_t launch_permute_mixed(int prec, int dtype, const void *psi, void *out, const MixedDesc &md, int conj,
                                hipStream_t st) {
    const int64_t R = md.d[0] * md.d[1];
    const int64_t nst = brick_stages(prec, md.d[2]);
    dim3 grid(grid_for(brick_rows(R) * nst * brick_epr(prec), 256 * 4, 65535 * 8)), block(256);
#define TNSLQ_PM(P, T) hipLaunchKernelGGL((k_permute_mixed<P, T>), grid, block, 0, st, psi, out, md, nst, conj)
    if (dtype == TNSLQ_C128) {
        switch (prec) {
            case TNSLQ_FP64: TNSLQ_PM(TNSLQ_FP64, TNSLQ_C128); break;
            case TNSLQ_FP32: TNSLQ_PM(TNSLQ_FP32, TNSLQ_C128); break;
            case TNSLQ_BF16X3: TNSLQ_PM(TNSLQ_BF16X3, TNSLQ_C128); break;
            default: TNSLQ_PM(TNSLQ_BF16X6, TNSLQ_C128); break;
        }
    } else {
        switch (prec) {
            case TNSLQ_FP64: TNSLQ_PM(TNSLQ_FP64, TNSLQ_C64); break;
            case TNSLQ_FP32: TNSLQ_PM(TNSLQ_FP32, TNSLQ_C64); break;
            case TNSLQ_BF16X3: TNSLQ_PM(TNSLQ_BF16X3, TNSLQ_C64); break;
            default: TNSLQ_PM(TNSLQ_BF16X6, TNSLQ_C64); break;
        }
    }
#undef TNSLQ_PM
    return hipGetLastError();
}

hipError_t launch_pt_bricks(int prec, int accfp64, const void *C, int64_t n, int64_t dB, void *rho, int64_t rho_nst,
                            hipStream_t st) {
    if ((prec == TNSLQ_FP64) != (accfp64 != 0)) return hipErrorInvalidValue;
    dim3 grid(grid_for(brick_rows(n) * rho_nst * brick_epr(prec), 256 * 4, 65535 * 8)), block(256);
#define TNSLQ_PTB(P, A) \
    hipLaunchKernelGGL((k_pt_bricks<P, A>), grid, block, 0, st, (const A *)C, n, dB, rho, rho_nst)
    switch (prec) {
        case TNSLQ_FP64: TNSLQ_PTB(TNSLQ_FP64, double2); break;
        case TNSLQ_FP32: TNSLQ_PTB(TNSLQ_FP32, float2); break;
        case TNSLQ_BF16X3: TNSLQ_PTB(TNSLQ_BF16X3, float2); break;
        default: TNSLQ_PTB(TNSLQ_BF16X6, float2); break;
    }
#undef TNSLQ_PTB
    return hipGetLastError();
}

hipError_t launch_pt_dense(const double2 *C, int64_t n, int64_t dB, double2 *out, hipStream_t st) {
    dim3 grid(grid_for(n * n, 256 * 4, 65535 * 4)), block(256);
    hipLaunchKernelGGL(k_pt_dense, grid, block, 0, st, C, n, dB, out);
    return hipGetLastError();
}

hipError_t launch_load_vectors_plain(const double2 *X, int64_t dA, int64_t dB, int K, int swapped, double2 *Xs,
                                     hipStream_t st) {
    dim3 grid(grid_for(dA * dB, 256 * 8, 4096), K), block(256);
    hipLaunchKernelGGL(k_load_vectors_plain, grid, block, 0, st, X, dA, dB, swapped, Xs);
    return hipGetLastError();
}

}  // namespace tnslq
