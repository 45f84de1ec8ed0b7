// Complex "NT" contraction C = A * B^T on the BF16 matrix cores with the
// hi + lo split (three real products per real product: hi*hi + hi*lo +
// lo*hi) and FP32 accumulation.
//
// Complex products use four real MFMA chains per split term:
//   Re C += Re A Re B + (-Im A) Im B,   Im C += Re A Im B + Im A Re B,
// the sign of Im A applied by flipping BF16 sign bits in registers.
//
// Tiling (gfx950, wave64): a 256-thread block computes a 128 x 128 complex
// output tile; its four waves each own 64 x 64 (4 x 4 MFMA tiles of
// 16 x 16).  Per reduction step of 32 the block stages 128 x 32 elements of
// each of the four operand planes of A and of B in LDS (rows padded to 80
// bytes so that the 16-byte fragment reads of 16 consecutive rows fall in
// distinct banks) and prefetches the next step into registers while the
// current one is multiplied.  Blocks walk the output in groups of 16 tile
// rows so that concurrently resident blocks share their A and B tiles in the
// caches.
#include "tnslq_internal.h"

namespace tnslq {
namespace {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(4))) float f32x4;

constexpr int BM = 128, BN = 128, BK = 32;
constexpr int NPL = 4;                 // re_hi, re_lo, im_hi, im_lo
constexpr int ROWB = 80;               // LDS bytes per staged row (64 data + 16 pad)
constexpr int TILEB = BM * ROWB;       // LDS bytes per plane tile
constexpr int LDS_BYTES = 2 * NPL * TILEB;
constexpr int GROUP_M = 16;

__device__ inline bf16x8 as_bf16x8(uint4 v) { return __builtin_bit_cast(bf16x8, v); }
__device__ inline uint4 neg_bf16x8(uint4 v) {
    return make_uint4(v.x ^ 0x80008000u, v.y ^ 0x80008000u, v.z ^ 0x80008000u, v.w ^ 0x80008000u);
}

__global__ void __launch_bounds__(256, 1) k_cgemm_nt_bf16x3(GemmDesc g) {
    extern __shared__ __attribute__((aligned(16))) char lds[];
    char *As = lds;
    char *Bs = lds + NPL * TILEB;

    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int wm = wid >> 1, wn = wid & 1;

    // grouped tile order: block -> (split, row tile, column tile)
    const int64_t ntm = (g.M + BM - 1) / BM, ntn = (g.N + BN - 1) / BN;
    const int64_t per_split = ntm * ntn;
    const int64_t bid = blockIdx.x;
    const int s = (int)(bid / per_split);
    const int64_t t = bid % per_split;
    const int64_t group = t / (GROUP_M * ntn);
    const int64_t first_m = group * GROUP_M;
    const int64_t gsize = (ntm - first_m) < GROUP_M ? (ntm - first_m) : GROUP_M;
    const int64_t tm = first_m + (t % (GROUP_M * ntn)) % gsize;
    const int64_t tn = (t % (GROUP_M * ntn)) / gsize;
    const int64_t i0 = tm * BM, j0 = tn * BN;

    const int64_t klen = g.Kr / g.S;
    const int64_t kbeg = (int64_t)s * klen, kend = kbeg + klen;

    const uint16_t *A = (const uint16_t *)g.A;
    const uint16_t *B = (const uint16_t *)g.B;

    // global -> register staging: per plane, two 16-byte units of A and of B
    uint4 ra[NPL][2], rb[NPL][2];
    const int urow0 = tid >> 2, ucol = tid & 3;   // unit u = tid + 256 t: row = u / 4, unit = u % 4
    auto gload = [&](int64_t l0) {
#pragma unroll
        for (int tt = 0; tt < 2; ++tt) {
            const int row = urow0 + 64 * tt;
            const int64_t gi = i0 + row, gj = j0 + row;
#pragma unroll
            for (int p = 0; p < NPL; ++p) {
                ra[p][tt] = gi < g.M ? *(const uint4 *)(A + p * g.a_ps + gi * g.lda + l0 + 8 * ucol)
                                     : make_uint4(0, 0, 0, 0);
                rb[p][tt] = gj < g.N ? *(const uint4 *)(B + p * g.b_ps + gj * g.ldb + l0 + 8 * ucol)
                                     : make_uint4(0, 0, 0, 0);
            }
        }
    };
    auto lstore = [&]() {
#pragma unroll
        for (int tt = 0; tt < 2; ++tt) {
            const int row = urow0 + 64 * tt;
#pragma unroll
            for (int p = 0; p < NPL; ++p) {
                *(uint4 *)(As + p * TILEB + row * ROWB + 16 * ucol) = ra[p][tt];
                *(uint4 *)(Bs + p * TILEB + row * ROWB + 16 * ucol) = rb[p][tt];
            }
        }
    };

    f32x4 accr[4][4], acci[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            accr[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
            acci[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
        }

    const int frow = lane & 15, fk = lane >> 4;   // fragment row within a 16-row tile, k-unit
    gload(kbeg);
    for (int64_t l0 = kbeg; l0 < kend; l0 += BK) {
        __syncthreads();
        lstore();
        __syncthreads();
        if (l0 + BK < kend) gload(l0 + BK);

        uint4 fa[4][NPL], fb[4][NPL];
#pragma unroll
        for (int x = 0; x < 4; ++x) {
            const int ra_row = wm * 64 + x * 16 + frow;
            const int rb_row = wn * 64 + x * 16 + frow;
#pragma unroll
            for (int p = 0; p < NPL; ++p) {
                fa[x][p] = *(const uint4 *)(As + p * TILEB + ra_row * ROWB + 16 * fk);
                fb[x][p] = *(const uint4 *)(Bs + p * TILEB + rb_row * ROWB + 16 * fk);
            }
        }
        uint4 nai[4][2];
#pragma unroll
        for (int x = 0; x < 4; ++x) {
            nai[x][0] = neg_bf16x8(fa[x][2]);
            nai[x][1] = neg_bf16x8(fa[x][3]);
        }
        // split terms (p, q) in {(hi,hi), (hi,lo), (lo,hi)}
#pragma unroll
        for (int term = 0; term < 3; ++term) {
            const int p = term == 2 ? 1 : 0;
            const int q = term == 1 ? 1 : 0;
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    accr[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(fa[a][p]), as_bf16x8(fb[b][q]),
                                                                          accr[a][b], 0, 0, 0);
                    acci[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(fa[a][p]),
                                                                          as_bf16x8(fb[b][2 + q]), acci[a][b], 0, 0, 0);
                }
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    accr[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(nai[a][p]),
                                                                          as_bf16x8(fb[b][2 + q]), accr[a][b], 0, 0, 0);
                    acci[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(fa[a][2 + p]),
                                                                          as_bf16x8(fb[b][q]), acci[a][b], 0, 0, 0);
                }
        }
    }

    // epilogue: lane holds rows 4 * (lane / 16) + r of column lane % 16
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t i = i0 + wm * 64 + a * 16 + 4 * fk + r;
                const int64_t j = j0 + wn * 64 + b * 16 + frow;
                if (i >= g.M || j >= g.N) continue;
                const int64_t addr = (j / g.cnb) * g.cbs + i * g.ldc + (j % g.cnb);
                const float vr = accr[a][b][r], vi = acci[a][b][r];
                if (g.out_mode == 0)
                    store_planes_f<TNSLQ_BF16X3>(g.C, g.c_ps, addr, vr, vi);
                else
                    ((float2 *)g.C)[s * g.c_split + addr] = make_float2(vr, vi);
            }
}

}  // namespace

// Shapes the matrix-core kernel takes: reduction per split a multiple of 32
// and 16-byte aligned rows.
bool gemm_bf16x3_supported(const GemmDesc &g) {
    const int64_t klen = g.Kr / g.S;
    return g.Kr % g.S == 0 && klen % BK == 0 && g.lda % 8 == 0 && g.ldb % 8 == 0 && g.a_ps % 8 == 0 &&
           g.b_ps % 8 == 0 && ((uintptr_t)g.A % 16) == 0 && ((uintptr_t)g.B % 16) == 0;
}

hipError_t launch_gemm_bf16x3(const GemmDesc &g, hipStream_t st) {
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute((const void *)k_cgemm_nt_bf16x3, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           LDS_BYTES);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    const int64_t nblocks = ((g.M + BM - 1) / BM) * ((g.N + BN - 1) / BN) * g.S;
    if (nblocks < 1 || nblocks > 0x7fffffff) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL(k_cgemm_nt_bf16x3, dim3((unsigned)nblocks), dim3(256), LDS_BYTES, st, g);
    return hipGetLastError();
}

}  // namespace tnslq
