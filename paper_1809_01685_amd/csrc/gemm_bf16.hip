// Complex "NT" contraction C = A * B^T on the BF16 matrix cores with the
// hi + lo split (three real products per real product: hi*hi + hi*lo +
// lo*hi) and FP32 accumulation.
//
// Complex products use four real MFMA chains per split term:
//   Re C += Re A Re B + (-Im A) Im B,   Im C += Re A Im B + Im A Re B,
// the sign of Im A applied by flipping BF16 sign bits in registers.
//
// Tiling (gfx950, wave64): a block computes a 128 x 128 complex output tile
// with WAVES_M x WAVES_N waves, each owning TM x TN MFMA tiles of 16 x 16
// (v_mfma_f32_16x16x32_bf16).  Per reduction step of 32 the block stages
// 128 x 32 elements of each of the four operand planes of A and of B in LDS,
// double buffered: while the waves multiply step i out of one buffer, step
// i+1 (loaded from global memory one step earlier) is written to the other and
// step i+2 is loaded into registers, with one barrier per step.  Rows are 64
// bytes; the four 16-byte units of a row are XOR-swizzled by
// ((row >> 1) ^ (row >> 2)) & 3 so that the fragment reads of 8 or 16
// consecutive rows hit distinct banks.
//
// Block order: the hardware deals blocks to the eight XCDs round robin, so
// block b is renumbered to give XCD b % 8 a contiguous range of output tiles,
// walked in groups of 4 tile rows; the ~32 blocks resident on one XCD then
// cover a compact 4 x 8 patch of tiles and share their A and B tiles in that
// XCD's L2.
#include "tnslq_internal.h"

namespace tnslq {
namespace {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(4))) float f32x4;

constexpr int BM = 128, BN = 128, BK = 32;
constexpr int NPL = 4;                   // re_hi, re_lo, im_hi, im_lo
constexpr int ROWB = 64;                 // LDS bytes per staged row
constexpr int TILEB = BM * ROWB;         // LDS bytes per plane tile
constexpr int STAGEB = 2 * NPL * TILEB;  // A and B planes of one reduction step
constexpr int LDS_BYTES = 2 * STAGEB;    // double buffered
constexpr int GROUP_M = 4;

// Block shape: 8 waves (2 per SIMD, so one wave's LDS waits overlap the
// other's matrix instructions), each owning 64 x 32 outputs.
constexpr int WAVES_M = 2, WAVES_N = 4;
constexpr int TM = BM / (16 * WAVES_M), TN = BN / (16 * WAVES_N);
constexpr int NT = 64 * WAVES_M * WAVES_N;
constexpr int UPT = BM * 4 / NT;         // 16-byte staging units per thread per plane

__device__ inline bf16x8 as_bf16x8(uint4 v) { return __builtin_bit_cast(bf16x8, v); }
__device__ inline uint4 neg_bf16x8(uint4 v) {
    return make_uint4(v.x ^ 0x80008000u, v.y ^ 0x80008000u, v.z ^ 0x80008000u, v.w ^ 0x80008000u);
}

// byte offset of 16-byte unit `u` of staged row `row` within a plane tile
__device__ inline int loff(int row, int u) { return row * ROWB + 16 * (u ^ (((row >> 1) ^ (row >> 2)) & 3)); }

// Main reduction loop over [kbeg, kend) for the block's output tile at
// (i0, j0).  FULL = the tile lies inside C, so no operand row needs zeroing.
template <bool FULL>
__device__ __forceinline__ void mainloop(const GemmDesc &g, char *lds, int64_t i0, int64_t j0, int64_t kbeg,
                                         int64_t kend, f32x4 (&accr)[TM][TN], f32x4 (&acci)[TM][TN]) {
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int wm = wid / WAVES_N, wn = wid % WAVES_N;
    const uint16_t *A = (const uint16_t *)g.A;
    const uint16_t *B = (const uint16_t *)g.B;

    // global -> register staging: per plane, UPT 16-byte units of A and of B.
    // Rows past the edge of A or B read a clamped in-range row and are zeroed.
    uint4 ra[NPL][UPT], rb[NPL][UPT];
    const int urow0 = tid >> 2, ucol = tid & 3;   // unit u = tid + NT t: row = u / 4, unit = u % 4
    const uint16_t *arow[UPT], *brow[UPT];
    bool aok[UPT], bok[UPT];
#pragma unroll
    for (int tt = 0; tt < UPT; ++tt) {
        const int row = urow0 + (NT / 4) * tt;
        const int64_t gi = i0 + row, gj = j0 + row;
        aok[tt] = FULL || gi < g.M;
        bok[tt] = FULL || gj < g.N;
        arow[tt] = A + (gi < g.M ? gi : g.M - 1) * g.lda + 8 * ucol;
        brow[tt] = B + (gj < g.N ? gj : g.N - 1) * g.ldb + 8 * ucol;
    }
    auto gload = [&](int64_t l0) {
#pragma unroll
        for (int tt = 0; tt < UPT; ++tt) {
#pragma unroll
            for (int p = 0; p < NPL; ++p) {
                uint4 va = *(const uint4 *)(arow[tt] + p * g.a_ps + l0);
                uint4 vb = *(const uint4 *)(brow[tt] + p * g.b_ps + l0);
                if constexpr (FULL) {
                    ra[p][tt] = va;
                    rb[p][tt] = vb;
                } else {
                    ra[p][tt] = aok[tt] ? va : make_uint4(0, 0, 0, 0);
                    rb[p][tt] = bok[tt] ? vb : make_uint4(0, 0, 0, 0);
                }
            }
        }
    };
    auto lstore = [&](int buf) {
        char *As = lds + buf * STAGEB, *Bs = As + NPL * TILEB;
#pragma unroll
        for (int tt = 0; tt < UPT; ++tt) {
            const int off = loff(urow0 + (NT / 4) * tt, ucol);
#pragma unroll
            for (int p = 0; p < NPL; ++p) {
                *(uint4 *)(As + p * TILEB + off) = ra[p][tt];
                *(uint4 *)(Bs + p * TILEB + off) = rb[p][tt];
            }
        }
    };

    const int frow = lane & 15, fk = lane >> 4;   // fragment row within a 16-row tile, k-unit
    gload(kbeg);
    lstore(0);
    if (kbeg + BK < kend) gload(kbeg + BK);
    __syncthreads();
    int buf = 0;
    for (int64_t l0 = kbeg; l0 < kend; l0 += BK, buf ^= 1) {
        const char *As = lds + buf * STAGEB, *Bs = As + NPL * TILEB;
        uint4 fa[TM][NPL], fb[TN][NPL];
#pragma unroll
        for (int x = 0; x < TM; ++x) {
            const int oa = loff(wm * TM * 16 + x * 16 + frow, fk);
#pragma unroll
            for (int p = 0; p < NPL; ++p) fa[x][p] = *(const uint4 *)(As + p * TILEB + oa);
        }
#pragma unroll
        for (int x = 0; x < TN; ++x) {
            const int ob = loff(wn * TN * 16 + x * 16 + frow, fk);
#pragma unroll
            for (int p = 0; p < NPL; ++p) fb[x][p] = *(const uint4 *)(Bs + p * TILEB + ob);
        }
        if (l0 + BK < kend) {
            lstore(buf ^ 1);
            if (l0 + 2 * BK < kend) gload(l0 + 2 * BK);
        }
        uint4 nai[TM][2];
#pragma unroll
        for (int x = 0; x < TM; ++x) {
            nai[x][0] = neg_bf16x8(fa[x][2]);
            nai[x][1] = neg_bf16x8(fa[x][3]);
        }
        // split terms (p, q) in {(hi,hi), (hi,lo), (lo,hi)}
#pragma unroll
        for (int term = 0; term < 3; ++term) {
            const int p = term == 2 ? 1 : 0;
            const int q = term == 1 ? 1 : 0;
#pragma unroll
            for (int a = 0; a < TM; ++a)
#pragma unroll
                for (int b = 0; b < TN; ++b) {
                    accr[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(fa[a][p]), as_bf16x8(fb[b][q]),
                                                                          accr[a][b], 0, 0, 0);
                    acci[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(fa[a][p]),
                                                                          as_bf16x8(fb[b][2 + q]), acci[a][b], 0, 0, 0);
                }
#pragma unroll
            for (int a = 0; a < TM; ++a)
#pragma unroll
                for (int b = 0; b < TN; ++b) {
                    accr[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(nai[a][p]),
                                                                          as_bf16x8(fb[b][2 + q]), accr[a][b], 0, 0, 0);
                    acci[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(fa[a][2 + p]),
                                                                          as_bf16x8(fb[b][q]), acci[a][b], 0, 0, 0);
                }
        }
        __syncthreads();
    }
}

__global__ void __launch_bounds__(NT, 1) k_cgemm_nt_bf16x3(GemmDesc g) {
    extern __shared__ __attribute__((aligned(16))) char lds[];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int wm = wid / WAVES_N, wn = wid % WAVES_N;

    // grouped tile order: block -> (split, row tile, column tile)
    const int64_t ntm = (g.M + BM - 1) / BM, ntn = (g.N + BN - 1) / BN;
    const int64_t per_split = ntm * ntn;
    int64_t bid = blockIdx.x;
    if (gridDim.x % 8 == 0) {
        // blocks are dealt to the 8 XCDs round robin: give each XCD a
        // contiguous range of tiles so its resident blocks share operands in L2
        bid = (bid % 8) * (gridDim.x / 8) + bid / 8;
    }
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

    f32x4 accr[TM][TN], acci[TM][TN];
#pragma unroll
    for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < TN; ++b) {
            accr[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
            acci[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
        }
    if (i0 + BM <= g.M && j0 + BN <= g.N)
        mainloop<true>(g, lds, i0, j0, kbeg, kend, accr, acci);
    else
        mainloop<false>(g, lds, i0, j0, kbeg, kend, accr, acci);

    // epilogue: lane holds rows 4 * (lane / 16) + r of column lane % 16
    const int frow = lane & 15, fk = lane >> 4;
#pragma unroll
    for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < TN; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t i = i0 + wm * TM * 16 + a * 16 + 4 * fk + r;
                const int64_t j = j0 + wn * TN * 16 + b * 16 + frow;
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
    hipLaunchKernelGGL(k_cgemm_nt_bf16x3, dim3((unsigned)nblocks), dim3(NT), LDS_BYTES, st, g);
    return hipGetLastError();
}

}  // namespace tnslq
