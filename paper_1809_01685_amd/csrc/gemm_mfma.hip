// Complex "NT" contraction C = A * B^T on the matrix cores (gfx950), for the
// two contractions of Sec. V Eq. 4, in three arithmetics:
//   BF16X3  operands split as hi + lo BF16 pieces, three real products per
//           real product (hi*hi + hi*lo + lo*hi), v_mfma_f32_16x16x32_bf16,
//           FP32 accumulation;
//   BF16X6  hi + mid + lo pieces, the six products of pieces (p, q) with
//           p + q < 3, FP32 accumulation restarted every 64 terms
//           (k_cgemm_bf16x6, 128 x 64 output tiles);
//   FP32    v_mfma_f32_16x16x4_f32 with FP32 accumulation, the matrix-core
//           sums flushed every 64 reduction terms into a second accumulator
//           so that no FP32 running sum grows past 64 terms;
//   FP64    v_mfma_f64_16x16x4_f64.
//
// Complex products use four real MFMA chains:
//   Re C += Re A Re B + (-Im A) Im B,   Im C += Re A Im B + Im A Re B,
// the sign of Im A applied by flipping sign bits in registers.
//
// Tiling (wave64): a block of 8 waves computes a 128 x 128 complex output
// tile, each wave 64 x 32 (4 x 2 MFMA tiles of 16 x 16), two waves per SIMD
// so that one wave's LDS waits overlap the other's matrix instructions.  A
// reduction step stages one brick of each operand (128 rows x 64 bytes per
// plane: 32 BF16, 16 FP32 or 8 FP64 reduction terms) in LDS: thread t copies
// bytes [16 t, 16 t + 16) of every plane, so each load instruction of the
// block reads 8 KiB of contiguous memory and lands at the same offset in LDS.
// Double buffered, one barrier per step.  For BF16 (k_cgemm_bf16x3_ra) the
// copy goes straight from global memory into LDS (global_load_lds_dwordx4:
// 16 bytes per lane, each wave 1 KiB of every plane tile), and a wave reads
// the next step's fragments while its matrix instructions run on the current
// ones; see the comment at that kernel.  FP32 and FP64 stage through
// registers: step i+1 (loaded one step earlier) is written to the other
// buffer and step i+2 is loaded into registers.  Bricks store the four
// 16-byte units of a row XOR-swizzled by ((row >> 1) ^ (row >> 2)) & 3, so
// the fragment reads of 8 or 16
// consecutive rows hit distinct banks.  Rows past the edge of C come from the
// bricks' row padding and their results are dropped; the reduction padding
// holds zeros.  Each lane's 16-byte fragment
// feeds one BF16 MFMA (8 terms), four FP32 MFMAs or two FP64 MFMAs; A and B
// fragments pair the same reduction terms, so the order in which the terms of
// a unit enter the sum does not matter.
//
// Block order: the hardware deals blocks to the eight XCDs round robin, so
// block b is renumbered to give XCD b % 8 a contiguous range of output tiles,
// walked in groups of 4 tile rows; the ~32 blocks resident on one XCD then
// cover a compact 4 x 8 patch of tiles and share their A and B tiles in that
// XCD's L2.
#include "operands.h"

#include <type_traits>

namespace tnslq {
namespace {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(4))) float f32x4;
typedef __attribute__((ext_vector_type(4))) double f64x4;

constexpr int BM = 128, BN = 128;
constexpr int ROWB = 64;                 // LDS bytes per staged row
constexpr int TILEB = BM * ROWB;         // LDS bytes per plane tile
constexpr int GROUP_M = 4;
constexpr int WAVES_M = 2, WAVES_N = 4;
constexpr int TM = BM / (16 * WAVES_M), TN = BN / (16 * WAVES_N);
constexpr int NT = 64 * WAVES_M * WAVES_N;
static_assert(BM == BRICK_ROWS && BN == BRICK_ROWS && ROWB == BRICK_ROW_BYTES, "one brick per operand per step");
static_assert(BM * ROWB / 16 == NT, "one 16-byte unit of every brick plane per thread");

template <int PREC> struct MP;
template <> struct MP<TNSLQ_BF16X3> {
    static constexpr int NPL = 4;        // re_hi, re_lo, im_hi, im_lo
    using acc = f32x4;
};
template <> struct MP<TNSLQ_BF16X6> {
    static constexpr int NPL = 6;        // re_hi, re_mid, re_lo, im_hi, im_mid, im_lo
    using acc = f32x4;
};
template <> struct MP<TNSLQ_FP32> {
    static constexpr int NPL = 2;
    using acc = f32x4;
};
template <> struct MP<TNSLQ_FP64> {
    static constexpr int NPL = 2;
    using acc = f64x4;
};
// a 16-byte unit of a brick row feeds one 16x16x32 BF16 MFMA, four 16x16x4
// FP32 MFMAs or two 16x16x4 FP64 MFMAs per lane
static_assert(brick_epr(TNSLQ_BF16X3) == 32 && brick_epr(TNSLQ_FP32) == 16 && brick_epr(TNSLQ_FP64) == 8,
              "brick rows of 64 bytes");
static_assert(MP<TNSLQ_BF16X3>::NPL == planes_of(TNSLQ_BF16X3) && MP<TNSLQ_BF16X6>::NPL == planes_of(TNSLQ_BF16X6) &&
                  MP<TNSLQ_FP32>::NPL == planes_of(TNSLQ_FP32) && MP<TNSLQ_FP64>::NPL == planes_of(TNSLQ_FP64),
              "planes per brick");

template <int PREC> constexpr int stage_bytes() { return 2 * MP<PREC>::NPL * TILEB; }
template <int PREC> constexpr int lds_bytes() { return 2 * stage_bytes<PREC>(); }

__device__ inline bf16x8 as_bf16x8(uint4 v) { return __builtin_bit_cast(bf16x8, v); }
__device__ inline uint4 neg_bf16x8(uint4 v) {
    return make_uint4(v.x ^ 0x80008000u, v.y ^ 0x80008000u, v.z ^ 0x80008000u, v.w ^ 0x80008000u);
}
__device__ inline uint4 neg_f32x4(uint4 v) {
    return make_uint4(v.x ^ 0x80000000u, v.y ^ 0x80000000u, v.z ^ 0x80000000u, v.w ^ 0x80000000u);
}
__device__ inline uint4 neg_f64x2(uint4 v) { return make_uint4(v.x, v.y ^ 0x80000000u, v.z, v.w ^ 0x80000000u); }
__device__ inline float f32_at(uint4 v, int t) {
    return __uint_as_float(t == 0 ? v.x : (t == 1 ? v.y : (t == 2 ? v.z : v.w)));
}
__device__ inline double f64_at(uint4 v, int t) {
    return t == 0 ? __hiloint2double((int)v.y, (int)v.x) : __hiloint2double((int)v.w, (int)v.z);
}

// byte offset of 16-byte unit `u` of staged row `row` within a plane tile
__device__ inline int loff(int row, int u) { return row * ROWB + 16 * (u ^ brick_swizzle(row)); }

// One reduction stage of the complex product for the wave's TM x TN tiles.
template <int PREC>
__device__ __forceinline__ void stage_mfma(const uint4 (&fa)[TM][MP<PREC>::NPL], const uint4 (&fb)[TN][MP<PREC>::NPL],
                                           typename MP<PREC>::acc (&accr)[TM][TN],
                                           typename MP<PREC>::acc (&acci)[TM][TN]) {
    static_assert(PREC != TNSLQ_BF16X3, "split BF16 runs in k_cgemm_bf16x3_ra");
    if constexpr (PREC == TNSLQ_FP32) {
        uint4 nai[TM];
#pragma unroll
        for (int x = 0; x < TM; ++x) nai[x] = neg_f32x4(fa[x][1]);
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int a = 0; a < TM; ++a)
#pragma unroll
                for (int b = 0; b < TN; ++b) {
                    const float ar = f32_at(fa[a][0], t), ai = f32_at(fa[a][1], t), nai_t = f32_at(nai[a], t);
                    const float br = f32_at(fb[b][0], t), bi = f32_at(fb[b][1], t);
                    accr[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar, br, accr[a][b], 0, 0, 0);
                    accr[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(nai_t, bi, accr[a][b], 0, 0, 0);
                    acci[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar, bi, acci[a][b], 0, 0, 0);
                    acci[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(ai, br, acci[a][b], 0, 0, 0);
                }
    } else {
        uint4 nai[TM];
#pragma unroll
        for (int x = 0; x < TM; ++x) nai[x] = neg_f64x2(fa[x][1]);
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int a = 0; a < TM; ++a)
#pragma unroll
                for (int b = 0; b < TN; ++b) {
                    const double ar = f64_at(fa[a][0], t), ai = f64_at(fa[a][1], t), nai_t = f64_at(nai[a], t);
                    const double br = f64_at(fb[b][0], t), bi = f64_at(fb[b][1], t);
                    accr[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, br, accr[a][b], 0, 0, 0);
                    accr[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(nai_t, bi, accr[a][b], 0, 0, 0);
                    acci[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, bi, acci[a][b], 0, 0, 0);
                    acci[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai, br, acci[a][b], 0, 0, 0);
                }
    }
}

// Main reduction loop over bricks [sbeg, send) for the block's output tile at
// (i0, j0), accumulating into (outr, outi).
template <int PREC>
__device__ __forceinline__ void mainloop(const GemmDesc &g, char *lds, int64_t i0, int64_t j0, int64_t sbeg,
                                         int64_t send, typename MP<PREC>::acc (&outr)[TM][TN],
                                         typename MP<PREC>::acc (&outi)[TM][TN]) {
    using P = MP<PREC>;
    using Acc = typename P::acc;
    constexpr int NPL = P::NPL;
    constexpr int STAGEB = stage_bytes<PREC>();
    constexpr int BRICKB = NPL * TILEB;   // one brick, all planes
    // FP32 keeps a second accumulator: the matrix-core sums restart every
    // FLUSH stages (64 terms) and are added into (outr, outi).
    constexpr bool TWO_LEVEL = PREC == TNSLQ_FP32;
    constexpr int FLUSH = 4;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int wm = wid / WAVES_N, wn = wid % WAVES_N;
    const size_t blk = brick_block_bytes(PREC, g.nst);
    const char *ga = (const char *)g.A + (size_t)(i0 / BM) * blk + 16 * tid;
    const char *gb = (const char *)g.B + (size_t)(j0 / BN) * blk + 16 * tid;

    // global -> register staging: one 16-byte unit of A and of B per plane
    uint4 ra[NPL], rb[NPL];
    auto gload = [&](int64_t st) __attribute__((always_inline)) {
        const char *pa = ga + st * BRICKB, *pb = gb + st * BRICKB;
#pragma unroll
        for (int p = 0; p < NPL; ++p) {
            const uint4 va = *(const uint4 *)(pa + p * TILEB);
            const uint4 vb = *(const uint4 *)(pb + p * TILEB);
            ra[p] = va;
            rb[p] = vb;
        }
    };
    auto lstore = [&](int buf) __attribute__((always_inline)) {
        char *As = lds + buf * STAGEB + 16 * tid, *Bs = As + NPL * TILEB;
#pragma unroll
        for (int p = 0; p < NPL; ++p) {
            *(uint4 *)(As + p * TILEB) = ra[p];
            *(uint4 *)(Bs + p * TILEB) = rb[p];
        }
    };

    Acc accr[TM][TN], acci[TM][TN];
    auto zero = [&]() __attribute__((always_inline)) {
#pragma unroll
        for (int a = 0; a < TM; ++a)
#pragma unroll
            for (int b = 0; b < TN; ++b) {
                accr[a][b] = Acc{0, 0, 0, 0};
                acci[a][b] = Acc{0, 0, 0, 0};
            }
    };
    auto flush = [&]() __attribute__((always_inline)) {
#pragma unroll
        for (int a = 0; a < TM; ++a)
#pragma unroll
            for (int b = 0; b < TN; ++b) {
                outr[a][b] += accr[a][b];
                outi[a][b] += acci[a][b];
            }
    };
    zero();

    const int frow = lane & 15, fk = lane >> 4;   // fragment row within a 16-row tile, k-unit
    gload(sbeg);
    lstore(0);
    if (sbeg + 1 < send) gload(sbeg + 1);
    __syncthreads();
    int buf = 0, nstage = 0;
    for (int64_t st = sbeg; st < send; ++st, buf ^= 1) {
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
        if (st + 1 < send) {
            lstore(buf ^ 1);
            if (st + 2 < send) gload(st + 2);
        }
        stage_mfma<PREC>(fa, fb, accr, acci);
        if constexpr (TWO_LEVEL) {
            if (++nstage == FLUSH) {
                flush();
                zero();
                nstage = 0;
            }
        }
        __builtin_amdgcn_sched_barrier(0);
        __syncthreads();
    }
    if constexpr (TWO_LEVEL) {
        if (nstage) flush();
    } else {
#pragma unroll
        for (int a = 0; a < TM; ++a)
#pragma unroll
            for (int b = 0; b < TN; ++b) {
                outr[a][b] = accr[a][b];
                outi[a][b] = acci[a][b];
            }
    }
}

// Output tile (i0, j0) and reduction split s of block blockIdx.x: the
// hardware deals blocks to the XCDs round robin, so block b is renumbered to
// give XCD b % 8 a contiguous range, walked in groups of GROUP_M tile rows.
struct TileAt {
    int64_t i0, j0, sbeg, send;
    int s;
};
template <int TBN = BN>
__device__ inline TileAt tile_of(const GemmDesc &g) {
    const int64_t ntm = (g.M + BM - 1) / BM, ntn = (g.N + TBN - 1) / TBN;
    const int64_t per_split = ntm * ntn;
    int64_t bid = blockIdx.x;
    if (gridDim.x % 8 == 0) bid = (bid % 8) * (gridDim.x / 8) + bid / 8;
    TileAt r;
    r.s = (int)(bid / per_split);
    const int64_t t = bid % per_split;
    const int64_t group = t / (GROUP_M * ntn);
    const int64_t first_m = group * GROUP_M;
    const int64_t gsize = (ntm - first_m) < GROUP_M ? (ntm - first_m) : GROUP_M;
    r.i0 = (first_m + (t % (GROUP_M * ntn)) % gsize) * BM;
    r.j0 = ((t % (GROUP_M * ntn)) / gsize) * TBN;
    const int64_t per = g.nst / g.S;
    r.sbeg = (int64_t)r.s * per;
    r.send = r.sbeg + per;
    return r;
}

// Epilogue of a wave's WTM x WTN tiles of 16 x 16 whose first output row and
// column are (wi0, wj0): output register r of lane l holds column l % 16 and
// row 4 (l / 16) + r (FP32 accumulators) or row 4 r + l / 16 (FP64).
template <int PREC, int WTM, int WTN>
__device__ __forceinline__ void store_tiles(const GemmDesc &g, int s, int64_t wi0, int64_t wj0, int lane,
                                            const typename MP<PREC>::acc (&accr)[WTM][WTN],
                                            const typename MP<PREC>::acc (&acci)[WTM][WTN]) {
    const int frow = lane & 15, fk = lane >> 4;
    const int64_t cnb_mask = ((int64_t)1 << g.cnb_log2) - 1, cni_mask = ((int64_t)1 << g.cni_log2) - 1;
#pragma unroll
    for (int a = 0; a < WTM; ++a)
#pragma unroll
        for (int b = 0; b < WTN; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int orow = PREC == TNSLQ_FP64 ? 4 * r + fk : 4 * fk + r;
                const int64_t i = wi0 + a * 16 + orow;
                const int64_t j = wj0 + b * 16 + frow;
                if (i >= g.M || j >= g.N) continue;
                const int64_t jq = j >> g.cnb_log2, jr = j & cnb_mask;
                const auto vr = accr[a][b][r], vi = acci[a][b][r];
                if (g.out_mode == 0) {
                    const int64_t row = jq * g.crs + (i >> g.cni_log2);
                    const int64_t col = ((i & cni_mask) << g.cnb_log2) + jr;
                    const int64_t idx = brick_index(PREC, g.c_nst, row, col);
                    if constexpr (PREC == TNSLQ_FP64)
                        store_planes<PREC>(g.C, brick_ps(PREC), idx, vr, vi);
                    else
                        store_planes_f<PREC>(g.C, brick_ps(PREC), idx, vr, vi);
                } else {
                    const int64_t addr = s * g.c_split + jq * g.cbs + i * g.ldc + jr;
                    if constexpr (PREC == TNSLQ_FP64)
                        ((double2 *)g.C)[addr] = make_double2(vr, vi);
                    else
                        ((float2 *)g.C)[addr] = make_float2(vr, vi);
                }
            }
}

template <int PREC>
__global__ void __launch_bounds__(NT, 1) k_cgemm_nt_mfma(GemmDesc g) {
    using Acc = typename MP<PREC>::acc;
    extern __shared__ __attribute__((aligned(16))) char lds[];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int wm = wid / WAVES_N, wn = wid % WAVES_N;
    const TileAt tl = tile_of(g);

    Acc accr[TM][TN], acci[TM][TN];
#pragma unroll
    for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < TN; ++b) {
            accr[a][b] = Acc{0, 0, 0, 0};
            acci[a][b] = Acc{0, 0, 0, 0};
        }
    mainloop<PREC>(g, lds, tl.i0, tl.j0, tl.sbeg, tl.send, accr, acci);
    store_tiles<PREC, TM, TN>(g, tl.s, tl.i0 + wm * TM * 16, tl.j0 + wn * TN * 16, lane, accr, acci);
}

// ---------------------------------------------------------------------------
// BF16X3: the same block, waves and LDS stages as k_cgemm_nt_mfma, with the
// next stage's fragments read while the current stage's matrix instructions
// run.  B's fragments (32 registers per stage) are kept in two sets; A's are
// read one row of tiles at a time, each into the registers that row has just
// released, so that a wave waits for LDS only for A's last row.  The copy of
// the stage after next goes into the LDS buffer the current stage has left,
// right after the barrier that ends the previous stage; one barrier per
// stage, after which every wave's copy has landed and every wave holds its
// fragments.  The LDS buffers are four arrays (A and B of two stages), so
// that the compiler can tell a fragment read of one buffer from a copy into
// the other and does not make the read wait for the copy.  Reading ahead
// keeps the matrix cores 70-77% busy on the 30-qubit contractions, 2-3
// points more than reading each stage's fragments before its instructions;
// the clock, held by the chip's power limit, gives back most of that.

// the 24 matrix instructions of one row of tiles: A's fragment (re_hi,
// re_lo, im_hi, im_lo) against the TN B fragments.  Each accumulator takes,
// for the split terms (hi, hi), (hi, lo), (lo, hi) in turn, Re A Re B then
// (-Im A) Im B (real part), or Re A Im B then Im A Re B (imaginary part).
__device__ __forceinline__ void row_bf16x3(const uint4 (&fa)[4], const uint4 (&fb)[TN][4], f32x4 (&ar)[TN],
                                           f32x4 (&ai)[TN]) {
    const uint4 n0 = neg_bf16x8(fa[2]), n1 = neg_bf16x8(fa[3]);
#pragma unroll
    for (int term = 0; term < 3; ++term) {
        const int p = term == 2 ? 1 : 0;
        const int q = term == 1 ? 1 : 0;
#pragma unroll
        for (int b = 0; b < TN; ++b) {
            ar[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(fa[p]), as_bf16x8(fb[b][q]), ar[b], 0, 0, 0);
            ai[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(fa[p]), as_bf16x8(fb[b][2 + q]), ai[b], 0, 0, 0);
        }
#pragma unroll
        for (int b = 0; b < TN; ++b) {
            ar[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(p ? n1 : n0), as_bf16x8(fb[b][2 + q]), ar[b], 0,
                                                            0, 0);
            ai[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(fa[2 + p]), as_bf16x8(fb[b][q]), ai[b], 0, 0, 0);
        }
    }
}

typedef __attribute__((address_space(3))) void lds_void_t;
typedef __attribute__((address_space(1))) const void gbl_void_t;

__global__ void __launch_bounds__(NT, 1) k_cgemm_bf16x3_ra(GemmDesc g) {
    constexpr int NPL = 4;
    constexpr int BRICKB = NPL * TILEB;   // one brick, all planes: 32 KiB
    __shared__ __attribute__((aligned(16))) char ldsA0[BRICKB], ldsA1[BRICKB], ldsB0[BRICKB], ldsB1[BRICKB];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int wm = wid / WAVES_N, wn = wid % WAVES_N;
    const TileAt tl = tile_of(g);
    const int64_t sbeg = tl.sbeg, send = tl.send;

    // thread t copies bytes [16 t, 16 t + 16) of every plane tile; each
    // wave's load fills 1 KiB of LDS at the same offset.  Block-uniform
    // bases (scalar registers) plus one per-lane offset.
    const size_t blk = brick_block_bytes(TNSLQ_BF16X3, g.nst);
    const char *gA = (const char *)g.A + (size_t)(tl.i0 / BM) * blk;
    const char *gB = (const char *)g.B + (size_t)(tl.j0 / BN) * blk;
    const uint32_t toff = 16u * (uint32_t)tid;
    const int wofs = 1024 * __builtin_amdgcn_readfirstlane(wid);
    auto dma = [&](int64_t st, int buf) __attribute__((always_inline)) {
        const char *pa = gA + st * BRICKB, *pb = gB + st * BRICKB;
        char *As = (buf ? ldsA1 : ldsA0) + wofs, *Bs = (buf ? ldsB1 : ldsB0) + wofs;
#pragma unroll
        for (int p = 0; p < NPL; ++p) {
            __builtin_amdgcn_global_load_lds((gbl_void_t *)(pa + p * TILEB + toff), (lds_void_t *)(As + p * TILEB), 16,
                                             0, 0);
            __builtin_amdgcn_global_load_lds((gbl_void_t *)(pb + p * TILEB + toff), (lds_void_t *)(Bs + p * TILEB), 16,
                                             0, 0);
        }
    };
    const int frow = lane & 15, fk = lane >> 4;
    int oa[TM], ob[TN];
#pragma unroll
    for (int x = 0; x < TM; ++x) oa[x] = loff(wm * TM * 16 + x * 16 + frow, fk);
#pragma unroll
    for (int x = 0; x < TN; ++x) ob[x] = loff(wn * TN * 16 + x * 16 + frow, fk);
    auto read_a = [&](int buf, int x, uint4 (&f)[NPL]) __attribute__((always_inline)) {
        const char *As = (buf ? ldsA1 : ldsA0) + oa[x];
#pragma unroll
        for (int p = 0; p < NPL; ++p) f[p] = *(const uint4 *)(As + p * TILEB);
    };
    auto read_b = [&](int buf, uint4 (&f)[TN][NPL]) __attribute__((always_inline)) {
#pragma unroll
        for (int x = 0; x < TN; ++x) {
            const char *Bs = (buf ? ldsB1 : ldsB0) + ob[x];
#pragma unroll
            for (int p = 0; p < NPL; ++p) f[x][p] = *(const uint4 *)(Bs + p * TILEB);
        }
    };

    f32x4 accr[TM][TN], acci[TM][TN];
#pragma unroll
    for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < TN; ++b) {
            accr[a][b] = f32x4{0, 0, 0, 0};
            acci[a][b] = f32x4{0, 0, 0, 0};
        }
    uint4 fa[2][TM][NPL], fb[2][TN][NPL];

    // stages sbeg and sbeg + 1 into the two buffers, stage sbeg's fragments
    // into registers
    const int64_t last = send - 1;
    dma(sbeg, 0);
    dma(sbeg + 1 <= last ? sbeg + 1 : last, 1);
    __builtin_amdgcn_s_waitcnt(0x0f70);   // vmcnt(0)
    __syncthreads();
    read_b(0, fb[0]);
#pragma unroll
    for (int x = 0; x < TM; ++x) read_a(0, x, fa[0][x]);
    __builtin_amdgcn_s_waitcnt(0xc07f);   // lgkmcnt(0): buffer 0 may be refilled
    __syncthreads();

    // stage st (its fragments in set C, its operands in buffer C): stage
    // st + 1's fragments from buffer C ^ 1 into set C ^ 1, stage st + 2's
    // operands into buffer C (the last stage again at the end of the run)
    auto body = [&](auto cc, int64_t st) __attribute__((always_inline)) {
        constexpr int C = decltype(cc)::value, N = C ^ 1;
        read_b(N, fb[N]);
        __builtin_amdgcn_sched_barrier(0);
        dma(st + 2 <= last ? st + 2 : last, C);
        __builtin_amdgcn_sched_barrier(0);
        // A's row a of the next stage into the registers row a has just
        // released
#pragma unroll
        for (int a = 0; a < TM; ++a) {
            row_bf16x3(fa[C][a], fb[C], accr[a], acci[a]);
            __builtin_amdgcn_sched_barrier(0);
            read_a(N, a, fa[N][a]);
            __builtin_amdgcn_sched_barrier(0);
        }
        __builtin_amdgcn_s_waitcnt(0x0070);   // vmcnt(0) and lgkmcnt(0)
        __syncthreads();
    };
    int64_t st = sbeg;
    for (; st + 1 < send; st += 2) {
        body(std::integral_constant<int, 0>{}, st);
        body(std::integral_constant<int, 1>{}, st + 1);
    }
    if (st < send) body(std::integral_constant<int, 0>{}, st);
    store_tiles<TNSLQ_BF16X3, TM, TN>(g, tl.s, tl.i0 + wm * TM * 16, tl.j0 + wn * TN * 16, lane, accr, acci);
}

hipError_t launch_bf16x3_ra(const GemmDesc &g, hipStream_t st) {
    const int64_t nblocks = ((g.M + BM - 1) / BM) * ((g.N + BN - 1) / BN) * g.S;
    if (nblocks < 1 || nblocks > 0x7fffffff) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL(k_cgemm_bf16x3_ra, dim3((unsigned)nblocks), dim3(NT), 0, st, g);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// BF16X6: operands split as hi + mid + lo BF16 pieces (six planes per
// operand), the products of pieces (p, q) with p + q < 3, six per real
// product, in FP32 on the matrix cores.  Six planes of a 128 x 128 tile would
// take 96 KiB of LDS per step, so a block computes 128 x 64 outputs: A's
// brick (48 KiB) and the half of B's brick that holds its 64 rows (24 KiB)
// per step, double buffered in 144 KiB.  Eight waves (two per SIMD), each
// 32 x 32 outputs (2 x 2 tiles of 16 x 16): per step a wave issues 96 MFMAs,
// as in the three-piece kernel.  The matrix-core sums restart every two steps
// (64 terms) and are added into a second FP32 accumulator, so that no FP32
// running sum grows past 64 terms.
constexpr int X6_BN = 64, X6_WAVES_M = 4, X6_WAVES_N = 2;
constexpr int X6_TM = BM / (16 * X6_WAVES_M), X6_TN = X6_BN / (16 * X6_WAVES_N);
constexpr int X6_NT = 64 * X6_WAVES_M * X6_WAVES_N;
constexpr int X6_FLUSH = 2;
static_assert(X6_TM == 2 && X6_TN == 2 && X6_NT == 512, "32 x 32 per wave");

__global__ void __launch_bounds__(X6_NT, 1) k_cgemm_bf16x6(GemmDesc g) {
    constexpr int NPL = 6;
    constexpr int ABRICK = NPL * TILEB;        // A's brick, all planes: 48 KiB
    constexpr int BHALF = TILEB / 2;           // 64 rows of one plane of B: 4 KiB
    constexpr int BSTAGE = NPL * BHALF;        // 24 KiB
    __shared__ __attribute__((aligned(16))) char ldsA0[ABRICK], ldsA1[ABRICK], ldsB0[BSTAGE], ldsB1[BSTAGE];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int wm = wid / X6_WAVES_N, wn = wid % X6_WAVES_N;
    const TileAt tl = tile_of<X6_BN>(g);
    const int64_t sbeg = tl.sbeg, send = tl.send;

    const size_t blk = brick_block_bytes(TNSLQ_BF16X6, g.nst);
    const char *gA = (const char *)g.A + (size_t)(tl.i0 / BM) * blk;
    // B's rows j0 .. j0 + 63: the first or second half of every plane tile
    const char *gB = (const char *)g.B + (size_t)(tl.j0 / BN) * blk + ((tl.j0 % BN) / X6_BN) * BHALF;
    const int w = __builtin_amdgcn_readfirstlane(wid);
    const uint32_t loff16 = 16u * (uint32_t)lane;
    // A: thread t copies bytes [16 t, 16 t + 16) of each plane tile; B: wave
    // w copies the 1 KiB pieces w, w + 8 and w + 16 of the 24 (plane piece / 4,
    // quarter piece % 4 of its 4 KiB)
    auto dma = [&](int64_t st, int buf) __attribute__((always_inline)) {
        const char *pa = gA + st * ABRICK, *pb = gB + st * ABRICK;
        char *As = (buf ? ldsA1 : ldsA0) + 1024 * w, *Bs = buf ? ldsB1 : ldsB0;
#pragma unroll
        for (int p = 0; p < NPL; ++p)
            __builtin_amdgcn_global_load_lds((gbl_void_t *)(pa + p * TILEB + 1024 * w + loff16),
                                             (lds_void_t *)(As + p * TILEB), 16, 0, 0);
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const int piece = w + 8 * i, plane = piece / 4, quarter = piece % 4;
            __builtin_amdgcn_global_load_lds((gbl_void_t *)(pb + plane * TILEB + quarter * 1024 + loff16),
                                             (lds_void_t *)(Bs + plane * BHALF + quarter * 1024), 16, 0, 0);
        }
    };
    const int frow = lane & 15, fk = lane >> 4;
    int oa[X6_TM], ob[X6_TN];
#pragma unroll
    for (int x = 0; x < X6_TM; ++x) oa[x] = loff(wm * X6_TM * 16 + x * 16 + frow, fk);
#pragma unroll
    for (int x = 0; x < X6_TN; ++x) ob[x] = loff(wn * X6_TN * 16 + x * 16 + frow, fk);

    f32x4 accr[X6_TM][X6_TN], acci[X6_TM][X6_TN], outr[X6_TM][X6_TN], outi[X6_TM][X6_TN];
#pragma unroll
    for (int a = 0; a < X6_TM; ++a)
#pragma unroll
        for (int b = 0; b < X6_TN; ++b) {
            accr[a][b] = acci[a][b] = outr[a][b] = outi[a][b] = f32x4{0, 0, 0, 0};
        }
    const int64_t last = send - 1;
    dma(sbeg, 0);
    __builtin_amdgcn_s_waitcnt(0x0f70);   // vmcnt(0)
    __syncthreads();
    int nstage = 0;
    for (int64_t st = sbeg; st < send; ++st) {
        const int buf = (int)((st - sbeg) & 1);
        const char *As = buf ? ldsA1 : ldsA0, *Bs = buf ? ldsB1 : ldsB0;
        uint4 fa[X6_TM][NPL], fb[X6_TN][NPL];
#pragma unroll
        for (int x = 0; x < X6_TM; ++x)
#pragma unroll
            for (int p = 0; p < NPL; ++p) fa[x][p] = *(const uint4 *)(As + p * TILEB + oa[x]);
#pragma unroll
        for (int x = 0; x < X6_TN; ++x)
#pragma unroll
            for (int p = 0; p < NPL; ++p) fb[x][p] = *(const uint4 *)(Bs + p * BHALF + ob[x]);
        // every fragment read of the step is issued before the copy into
        // the other buffer
        __builtin_amdgcn_sched_barrier(0);
        dma(st + 1 <= last ? st + 1 : last, buf ^ 1);
        __builtin_amdgcn_sched_barrier(0);
        // pieces (p, q) with p + q < 3; Re C += Re A Re B + (-Im A) Im B,
        // Im C += Re A Im B + Im A Re B
#pragma unroll
        for (int pq = 0; pq < 6; ++pq) {
            const int p = pq < 3 ? 0 : (pq < 5 ? 1 : 2);
            const int q = pq < 3 ? pq : (pq < 5 ? pq - 3 : 0);
#pragma unroll
            for (int a = 0; a < X6_TM; ++a) {
                const uint4 na = neg_bf16x8(fa[a][3 + p]);
#pragma unroll
                for (int b = 0; b < X6_TN; ++b) {
                    accr[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(fa[a][p]), as_bf16x8(fb[b][q]),
                                                                          accr[a][b], 0, 0, 0);
                    acci[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(fa[a][p]),
                                                                          as_bf16x8(fb[b][3 + q]), acci[a][b], 0, 0, 0);
                    accr[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(na), as_bf16x8(fb[b][3 + q]),
                                                                          accr[a][b], 0, 0, 0);
                    acci[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(fa[a][3 + p]),
                                                                          as_bf16x8(fb[b][q]), acci[a][b], 0, 0, 0);
                }
            }
        }
        if (++nstage == X6_FLUSH) {
#pragma unroll
            for (int a = 0; a < X6_TM; ++a)
#pragma unroll
                for (int b = 0; b < X6_TN; ++b) {
                    outr[a][b] += accr[a][b];
                    outi[a][b] += acci[a][b];
                    accr[a][b] = acci[a][b] = f32x4{0, 0, 0, 0};
                }
            nstage = 0;
        }
        __builtin_amdgcn_sched_barrier(0);
        __builtin_amdgcn_s_waitcnt(0x0070);   // vmcnt(0) and lgkmcnt(0)
        __syncthreads();
    }
    if (nstage) {
#pragma unroll
        for (int a = 0; a < X6_TM; ++a)
#pragma unroll
            for (int b = 0; b < X6_TN; ++b) {
                outr[a][b] += accr[a][b];
                outi[a][b] += acci[a][b];
            }
    }
    store_tiles<TNSLQ_BF16X6, X6_TM, X6_TN>(g, tl.s, tl.i0 + wm * X6_TM * 16, tl.j0 + wn * X6_TN * 16, lane, outr,
                                            outi);
}

hipError_t launch_bf16x6(const GemmDesc &g, hipStream_t st) {
    const int64_t nblocks = ((g.M + BM - 1) / BM) * ((g.N + X6_BN - 1) / X6_BN) * g.S;
    if (nblocks < 1 || nblocks > 0x7fffffff) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL(k_cgemm_bf16x6, dim3((unsigned)nblocks), dim3(X6_NT), 0, st, g);
    return hipGetLastError();
}

template <int PREC>
hipError_t launch(const GemmDesc &g, hipStream_t st) {
    if constexpr (PREC == TNSLQ_BF16X3) {
        return launch_bf16x3_ra(g, st);
    } else {
        static bool attr_set = false;
        if (!attr_set) {
            hipError_t e = hipFuncSetAttribute((const void *)k_cgemm_nt_mfma<PREC>,
                                               hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes<PREC>());
            if (e != hipSuccess) return e;
            attr_set = true;
        }
        const int64_t nblocks = ((g.M + BM - 1) / BM) * ((g.N + BN - 1) / BN) * g.S;
        if (nblocks < 1 || nblocks > 0x7fffffff) return hipErrorInvalidConfiguration;
        hipLaunchKernelGGL(k_cgemm_nt_mfma<PREC>, dim3((unsigned)nblocks), dim3(NT), lds_bytes<PREC>(), st, g);
        return hipGetLastError();
    }
}

template <int PREC>
bool supported(const GemmDesc &g) {
    return g.S >= 1 && g.nst % g.S == 0 && ((uintptr_t)g.A % 16) == 0 && ((uintptr_t)g.B % 16) == 0;
}

}  // namespace

// Whether the matrix-core kernel takes this contraction: BF16X3, BF16X6, FP32
// or FP64 bricks, the bricks divided evenly between the splits.
bool gemm_mfma_supported(int prec, const GemmDesc &g) {
    switch (prec) {
        case TNSLQ_BF16X3: return supported<TNSLQ_BF16X3>(g);
        case TNSLQ_BF16X6: return supported<TNSLQ_BF16X6>(g);
        case TNSLQ_FP32: return supported<TNSLQ_FP32>(g);
        case TNSLQ_FP64: return supported<TNSLQ_FP64>(g);
        default: return false;
    }
}

hipError_t launch_gemm_mfma(int prec, const GemmDesc &g, hipStream_t st) {
    switch (prec) {
        case TNSLQ_BF16X3: return launch<TNSLQ_BF16X3>(g, st);
        case TNSLQ_BF16X6: return launch_bf16x6(g, st);
        case TNSLQ_FP32: return launch<TNSLQ_FP32>(g, st);
        case TNSLQ_FP64: return launch<TNSLQ_FP64>(g, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace tnslq
