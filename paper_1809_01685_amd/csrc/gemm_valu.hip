// Complex "NT" contraction C = A * B^T on the vector ALUs, over the same
// brick operands as the matrix-core kernel.
//
// Serves shapes the matrix-core kernels do not take (bricks not divided
// evenly between the splits, unaligned operands) and works for every
// precision, including the six-piece BF16 split (hi/mid/lo, the products with
// p + q < 3 formed in FP32).  Sums run in blocks of one LDS tile (16 terms), blocks added into
// a second accumulator.
#include "tnslq_internal.h"

namespace tnslq {
namespace {

template <int PREC> struct Pol;
template <> struct Pol<TNSLQ_FP64> { using T = double; static constexpr int NP = 1; };
template <> struct Pol<TNSLQ_FP32> { using T = float; static constexpr int NP = 1; };
template <> struct Pol<TNSLQ_BF16X3> { using T = float; static constexpr int NP = 2; };
template <> struct Pol<TNSLQ_BF16X6> { using T = float; static constexpr int NP = 3; };

template <int PREC> struct Elem {
    typename Pol<PREC>::T re[Pol<PREC>::NP], im[Pol<PREC>::NP];
};

template <int PREC>
__device__ inline Elem<PREC> load_elem(const void *base, int64_t ps, int64_t idx, bool valid) {
    Elem<PREC> e;
    constexpr int NP = Pol<PREC>::NP;
    if (!valid) {
#pragma unroll
        for (int p = 0; p < NP; ++p) e.re[p] = e.im[p] = 0;
        return e;
    }
    if constexpr (PREC == TNSLQ_FP64) {
        const double *b = (const double *)base;
        e.re[0] = b[idx];
        e.im[0] = b[ps + idx];
    } else if constexpr (PREC == TNSLQ_FP32) {
        const float *b = (const float *)base;
        e.re[0] = b[idx];
        e.im[0] = b[ps + idx];
    } else {
        const uint16_t *b = (const uint16_t *)base;
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            e.re[p] = bf16_to_f32(b[p * ps + idx]);
            e.im[p] = bf16_to_f32(b[(NP + p) * ps + idx]);
        }
    }
    return e;
}

// Products kept for each split: every (p, q) with p + q < NP.
template <int PREC, typename T>
__device__ inline void cmac(const Elem<PREC> &a, const Elem<PREC> &b, T &re, T &im) {
    constexpr int NP = Pol<PREC>::NP;
#pragma unroll
    for (int p = 0; p < NP; ++p)
#pragma unroll
        for (int q = 0; q < NP - p; ++q) {
            re += a.re[p] * b.re[q] - a.im[p] * b.im[q];
            im += a.re[p] * b.im[q] + a.im[p] * b.re[q];
        }
}

constexpr int BM = 64, BN = 64, BK = 16;

template <int PREC>
__global__ void __launch_bounds__(256) k_cgemm_nt_valu(GemmDesc g) {
    using T = typename Pol<PREC>::T;
    __shared__ Elem<PREC> As[BK][BM + 1];
    __shared__ Elem<PREC> Bs[BK][BN + 1];

    const int tid = threadIdx.x;
    const int tx = tid % 16, ty = tid / 16;
    // flat grid: block b -> (split s, row tile, column tile), column fastest
    const int64_t ntn = (g.N + BN - 1) / BN, ntm = (g.M + BM - 1) / BM;
    const int64_t bid = blockIdx.x;
    const int64_t tn = bid % ntn, tm = (bid / ntn) % ntm;
    const int s = (int)(bid / (ntn * ntm));
    const int64_t i0 = tm * BM;
    const int64_t j0 = tn * BN;
    // split s covers bricks [s nst / S, (s + 1) nst / S) of the reduction
    constexpr int EPR = brick_epr(PREC);
    const int64_t per = g.nst / g.S;
    const int64_t kbeg = s * per * EPR;
    const int64_t kend = (kbeg + per * EPR) < g.Kr ? (kbeg + per * EPR) : g.Kr;

    T tot_re[4][4], tot_im[4][4];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) tot_re[r][c] = tot_im[r][c] = 0;

    for (int64_t l0 = kbeg; l0 < kend; l0 += BK) {
        // stage A and B tiles: element e -> (row e / BK, l e % BK)
#pragma unroll
        for (int t = 0; t < (BM * BK) / 256; ++t) {
            const int e = tid + t * 256;
            const int row = e / BK, l = e % BK;
            const int64_t gi = i0 + row, gl = l0 + l;
            As[l][row] = load_elem<PREC>(g.A, brick_ps(PREC), brick_index(PREC, g.nst, gi, gl), gi < g.M && gl < kend);
            const int64_t gj = j0 + row;
            Bs[l][row] = load_elem<PREC>(g.B, brick_ps(PREC), brick_index(PREC, g.nst, gj, gl), gj < g.N && gl < kend);
        }
        __syncthreads();
        T blk_re[4][4], blk_im[4][4];
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int c = 0; c < 4; ++c) blk_re[r][c] = blk_im[r][c] = 0;
#pragma unroll 4
        for (int l = 0; l < BK; ++l) {
            Elem<PREC> a[4], b[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) a[r] = As[l][ty + 16 * r];
#pragma unroll
            for (int c = 0; c < 4; ++c) b[c] = Bs[l][tx + 16 * c];
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int c = 0; c < 4; ++c) cmac<PREC>(a[r], b[c], blk_re[r][c], blk_im[r][c]);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                tot_re[r][c] += blk_re[r][c];
                tot_im[r][c] += blk_im[r][c];
            }
        __syncthreads();
    }

#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int64_t i = i0 + ty + 16 * r;
        if (i >= g.M) continue;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int64_t j = j0 + tx + 16 * c;
            if (j >= g.N) continue;
            const int64_t jq = j >> g.cnb_log2, jr = j & (((int64_t)1 << g.cnb_log2) - 1);
            if (g.out_mode == 0) {
                const int64_t row = jq * g.crs + (i >> g.cni_log2);
                const int64_t col = ((i & (((int64_t)1 << g.cni_log2) - 1)) << g.cnb_log2) + jr;
                const int64_t idx = brick_index(PREC, g.c_nst, row, col);
                if constexpr (PREC == TNSLQ_FP64)
                    store_planes<PREC>(g.C, brick_ps(PREC), idx, tot_re[r][c], tot_im[r][c]);
                else
                    store_planes_f<PREC>(g.C, brick_ps(PREC), idx, tot_re[r][c], tot_im[r][c]);
            } else {
                const int64_t addr = s * g.c_split + jq * g.cbs + i * g.ldc + jr;
                if constexpr (PREC == TNSLQ_FP64)
                    ((double2 *)g.C)[addr] = make_double2(tot_re[r][c], tot_im[r][c]);
                else
                    ((float2 *)g.C)[addr] = make_float2(tot_re[r][c], tot_im[r][c]);
            }
        }
    }
}

}  // namespace

hipError_t launch_gemm_valu(int prec, const GemmDesc &g, hipStream_t st) {
    const int64_t nblocks = ((g.N + BN - 1) / BN) * ((g.M + BM - 1) / BM) * g.S;
    if (nblocks < 1 || nblocks > 0x7fffffff) return hipErrorInvalidConfiguration;
    dim3 grid((unsigned)nblocks), block(256);
    switch (prec) {
        case TNSLQ_FP64: hipLaunchKernelGGL(k_cgemm_nt_valu<TNSLQ_FP64>, grid, block, 0, st, g); break;
        case TNSLQ_FP32: hipLaunchKernelGGL(k_cgemm_nt_valu<TNSLQ_FP32>, grid, block, 0, st, g); break;
        case TNSLQ_BF16X3: hipLaunchKernelGGL(k_cgemm_nt_valu<TNSLQ_BF16X3>, grid, block, 0, st, g); break;
        default: hipLaunchKernelGGL(k_cgemm_nt_valu<TNSLQ_BF16X6>, grid, block, 0, st, g); break;
    }
    return hipGetLastError();
}

hipError_t launch_gemm(int prec, const GemmDesc &g, hipStream_t st) {
    if (gemm_mfma_supported(prec, g)) return launch_gemm_mfma(prec, g, st);
    return launch_gemm_valu(prec, g, st);
}

}  // namespace tnslq
