// Complex "NT" contraction C = A * B^T on the matrix cores (gfx950), for the
// two contractions of Sec. V Eq. 4, in these arithmetics:
//   BF16X3  operands split as hi + lo BF16 pieces, three products of pieces
//           per real product (hi*hi + hi*lo + lo*hi), three real products per
//           complex product (see k_cgemm_bf16x3), v_mfma_f32_16x16x32_bf16,
//           FP32 accumulation;
//   BF16X6  hi + mid + lo pieces, the six products of pieces (p, q) with
//           p + q < 3, FP32 accumulation restarted every 64 terms
//           (k_cgemm_bf16x6, 128 x 64 output tiles);
//   FP32    v_mfma_f32_16x16x4_f32 with FP32 accumulation, the matrix-core
//           sums flushed every 64 reduction terms into a second accumulator
//           so that no FP32 running sum grows past 64 terms;
//   FP64    v_mfma_f64_16x16x4_f64.
//
// Complex products in BF16X6, FP32 and FP64 use four real MFMA chains:
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
// Double buffered, one barrier per step.  For BF16 (k_cgemm_bf16x3,
// k_cgemm_bf16x6) the copy goes straight from global memory into LDS
// (global_load_lds_dwordx4: 16 bytes per lane, each wave 1 KiB of a plane
// tile); k_cgemm_bf16x3 stages one pair of planes at a time and reads the next
// pair's fragments while its matrix instructions run on the current ones; see
// the comment at that kernel.  FP32 and FP64 stage through
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
    static constexpr int NPL = 6;        // re_hi, re_lo, im_hi, im_lo, sum_hi, sum_lo
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
    static_assert(PREC != TNSLQ_BF16X3, "split BF16 runs in k_cgemm_bf16x3");
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
// BF16X3: three real products per complex product (Gauss's form),
//   T1 = sum Re A Re B,  T2 = sum Im A Im B,  T3 = sum (Re A + Im A)(Re B + Im B),
//   Re C = T1 - T2,      Im C = T3 - T1 - T2,
// each real product split as hi*hi + hi*lo + lo*hi: 9 matrix instructions per
// pair of 16 x 16 tiles and reduction step instead of 12.  The operands carry
// Re + Im as a third pair of planes (operands.h), so a brick is three 16 KiB
// pairs (re, im, sum; hi and lo of 128 rows each) in the order of the three
// products.  Staging a whole brick of both operands twice would take 192 KiB
// of LDS; the kernel stages instead one pair of planes of each operand per
// "phase" (32 KiB), and the phases of a block's run of bricks are consecutive
// 16 KiB pieces of its rows of A and of B.  Same block, waves and tiles as
// k_cgemm_nt_mfma (128 x 128 outputs, 8 waves of 64 x 32); per phase a wave
// issues 24 matrix instructions into the accumulators of that phase's product.
// Pipeline over a ring of four LDS buffers (128 KiB): in phase ph the matrix
// instructions run on phase ph's fragments while, issued between them, a wave
// reads phase ph + 1's fragments from its buffer into the second register set
// and the block copies phase ph + 4 into the buffer phase ph has left (its
// fragments are in registers); one barrier ends the phase once phase ph + 2
// has landed (the copies of ph + 3 and ph + 4 stay in flight).  Issuing the
// reads and copies before the matrix instructions instead left the matrix
// cores idle after every barrier: 254 / 270 ms per launch against 244 / 244.
// The barrier is a bare s_barrier after explicit wait counts: __syncthreads
// would add a fence that waits for every copy in flight.  Buffers, register
// sets and accumulators are chosen at
// compile time (the LDS buffers are eight arrays, so that the compiler tells a
// fragment read of one buffer from a copy into another): the loop body is 12
// phases (4 bricks), and a run whose phase count is not a multiple of 12
// starts with the last 3, 6 or 9 phases of that body, so the loop itself has
// no branch (a branch around each phase's instructions cost 8%).  Against the
// four-product kernel on the 30-qubit contractions, launched alone on one box:
// 244 / 244 ms per launch against 283 / 282, 14% rather than 25%, the rest
// taken by the 1.5x bytes staged per step (with the copies left out the loop
// took 189 ms) and the power they cost under the chip's power limit.
typedef __attribute__((address_space(3))) void lds_void_t;
typedef __attribute__((address_space(1))) const void gbl_void_t;

constexpr int PHB = 2 * TILEB;    // one pair of planes of one operand: 16 KiB
constexpr int X3_BODY = 12;       // phases per loop iteration: lcm(2 sets, 3 products, 4 buffers)

template <int U, int END, typename F>
__device__ __forceinline__ void unroll_from(F &f) {
    if constexpr (U < END) {
        f(std::integral_constant<int, U>{});
        unroll_from<U + 1, END>(f);
    }
}

__global__ void __launch_bounds__(NT, 1) k_cgemm_bf16x3(GemmDesc g) {
    __shared__ __attribute__((aligned(16))) char lA0[PHB], lA1[PHB], lA2[PHB], lA3[PHB];
    __shared__ __attribute__((aligned(16))) char lB0[PHB], lB1[PHB], lB2[PHB], lB3[PHB];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int wm = wid / WAVES_N, wn = wid % WAVES_N;
    const TileAt tl = tile_of(g);
    // phases of this block's run of bricks (3 per brick)
    const int64_t p0 = 3 * tl.sbeg, pend = 3 * tl.send, plast = pend - 1;
    const size_t blk = brick_block_bytes(TNSLQ_BF16X3, g.nst);
    const char *gA = (const char *)g.A + (size_t)(tl.i0 / BM) * blk;
    const char *gB = (const char *)g.B + (size_t)(tl.j0 / BN) * blk;
    const uint32_t toff = 16u * (uint32_t)tid;
    const int wofs = 1024 * __builtin_amdgcn_readfirstlane(wid);
    auto bufA = [&](auto bb) -> char * {
        constexpr int B = decltype(bb)::value;
        return B == 0 ? lA0 : (B == 1 ? lA1 : (B == 2 ? lA2 : lA3));
    };
    auto bufB = [&](auto bb) -> char * {
        constexpr int B = decltype(bb)::value;
        return B == 0 ? lB0 : (B == 1 ? lB1 : (B == 2 ? lB2 : lB3));
    };
    // copy phase ph (the last phase again past the end of the run) into
    // buffer bb: thread t copies bytes [16 t, 16 t + 16) of both plane tiles
    // of A and of B
    auto dma = [&](int64_t ph, auto bb) __attribute__((always_inline)) {
        const int64_t q = ph <= plast ? ph : plast;
        const char *pa = gA + q * PHB, *pb = gB + q * PHB;
        char *As = bufA(bb) + wofs, *Bs = bufB(bb) + wofs;
#pragma unroll
        for (int p = 0; p < 2; ++p) {
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
    // fragments (hi, lo) of the wave's A and B tiles, two sets
    uint4 fa[2][TM][2], fb[2][TN][2];
    auto rd = [&](auto ss, auto bb) __attribute__((always_inline)) {
        constexpr int S = decltype(ss)::value;
        const char *As = bufA(bb), *Bs = bufB(bb);
#pragma unroll
        for (int x = 0; x < TM; ++x)
#pragma unroll
            for (int p = 0; p < 2; ++p) fa[S][x][p] = *(const uint4 *)(As + p * TILEB + oa[x]);
#pragma unroll
        for (int x = 0; x < TN; ++x)
#pragma unroll
            for (int p = 0; p < 2; ++p) fb[S][x][p] = *(const uint4 *)(Bs + p * TILEB + ob[x]);
    };
    // T1, T2, T3
    f32x4 t[3][TM][TN];
#pragma unroll
    for (int q = 0; q < 3; ++q)
#pragma unroll
        for (int a = 0; a < TM; ++a)
#pragma unroll
            for (int b = 0; b < TN; ++b) t[q][a][b] = f32x4{0, 0, 0, 0};

    // phase base + U of the loop body (U = 0 .. 11): fragments in set U % 2,
    // operands in buffer U % 4, product U % 3
    int64_t base = 0;
    auto phase = [&](auto uu) __attribute__((always_inline)) {
        constexpr int U = decltype(uu)::value;
        constexpr int C = U % 2, Q = U % 3;
        const int64_t ph = base + U;
        rd(std::integral_constant<int, C ^ 1>{}, std::integral_constant<int, (U + 1) % 4>{});
        dma(ph + 4, std::integral_constant<int, U % 4>{});
#pragma unroll
        for (int term = 0; term < 3; ++term) {
            const int p = term == 2 ? 1 : 0, q = term == 1 ? 1 : 0;
#pragma unroll
            for (int a = 0; a < TM; ++a)
#pragma unroll
                for (int b = 0; b < TN; ++b)
                    t[Q][a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(fa[C][a][p]), as_bf16x8(fb[C][b][q]),
                                                                         t[Q][a][b], 0, 0, 0);
        }
        // the matrix instructions start right after the barrier, the 12
        // fragment reads and the 4 copies issued one between each pair
        // (2 MFMA, then 12 x (LDS read, MFMA), 4 x (copy, MFMA), 6 MFMA)
        __builtin_amdgcn_sched_group_barrier(0x008, 2, 0);
#pragma unroll
        for (int i = 0; i < 12; ++i) {
            __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
            __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);
            __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
        }
        __builtin_amdgcn_sched_group_barrier(0x008, 6, 0);
        __builtin_amdgcn_sched_barrier(0);
        __builtin_amdgcn_s_waitcnt(0x0078);   // vmcnt(8): phase ph + 2 landed; lgkmcnt(0)
        __builtin_amdgcn_s_barrier();
        __builtin_amdgcn_sched_barrier(0);
    };
    // the run starts at body position U0 (0, 3, 6 or 9), so that it ends with
    // a whole body: phases p0 .. p0 + 3 into buffers U0 .. U0 + 3 (mod 4),
    // phase p0's fragments into set U0 % 2, then body positions U0 .. 11
    auto start = [&](auto u0) __attribute__((always_inline)) {
        constexpr int V = decltype(u0)::value;
        dma(p0, std::integral_constant<int, V % 4>{});
        dma(p0 + 1, std::integral_constant<int, (V + 1) % 4>{});
        dma(p0 + 2, std::integral_constant<int, (V + 2) % 4>{});
        dma(p0 + 3, std::integral_constant<int, (V + 3) % 4>{});
        __builtin_amdgcn_s_waitcnt(0x0f7c);   // vmcnt(12): phase p0 landed
        __builtin_amdgcn_s_barrier();
        __builtin_amdgcn_sched_barrier(0);
        rd(std::integral_constant<int, V % 2>{}, std::integral_constant<int, V % 4>{});
        __builtin_amdgcn_s_waitcnt(0x0078);   // vmcnt(8): phase p0 + 1 landed; lgkmcnt(0)
        __builtin_amdgcn_s_barrier();
        __builtin_amdgcn_sched_barrier(0);
        base = p0 - V;
        unroll_from<V, X3_BODY>(phase);
        base += X3_BODY;
    };
    const int u0 = (int)((X3_BODY - (pend - p0) % X3_BODY) % X3_BODY);
    switch (u0) {
        case 3: start(std::integral_constant<int, 3>{}); break;
        case 6: start(std::integral_constant<int, 6>{}); break;
        case 9: start(std::integral_constant<int, 9>{}); break;
        default: start(std::integral_constant<int, 0>{}); break;
    }
    for (; base < pend; base += X3_BODY) unroll_from<0, X3_BODY>(phase);

    f32x4 accr[TM][TN], acci[TM][TN];
#pragma unroll
    for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < TN; ++b) {
            accr[a][b] = t[0][a][b] - t[1][a][b];
            acci[a][b] = t[2][a][b] - t[0][a][b] - t[1][a][b];
        }
    if (g.out_mode != 0 || g.cnb_log2 < 3) {
        store_tiles<TNSLQ_BF16X3, TM, TN>(g, tl.s, tl.i0 + wm * TM * 16, tl.j0 + wn * TN * 16, lane, accr, acci);
        return;
    }
    // Output as bricks (the first contraction's intermediary), through LDS.
    // Per element the MFMA layout gives a lane one column and scattered rows,
    // so direct stores are 2-byte pieces (192 per lane; they cost 8% of the
    // launch).  Instead, one pair of planes at a time (re, im, re + im; hi and
    // lo) goes into LDS as [plane][row][column] and leaves in 16-byte units:
    // 8 consecutive columns j are 8 consecutive reduction terms of one brick
    // row when cnb >= 8.  Rows are taken in the order of their environment
    // index i % cni, so that a wave writes consecutive brick rows.  Staging
    // rows of 288 bytes (128 columns + 16 of padding) keep the 2-byte writes
    // of a wave's 4 row groups in distinct banks; plane p's rows 32 m .. 32 m
    // + 31 live in ring buffer 4 p + m (9 KiB of its 16).
    __builtin_amdgcn_s_waitcnt(0x0070);   // every copy (the clamped ones past the end) landed
    __syncthreads();
    constexpr int SROW = 288;
    auto sbase = [&](int pm) -> char * {
        return pm == 0 ? lA0
                       : (pm == 1 ? lA1
                                  : (pm == 2 ? lA2
                                             : (pm == 3 ? lA3 : (pm == 4 ? lB0 : (pm == 5 ? lB1 : (pm == 6 ? lB2 : lB3))))));
    };
    const int nB = g.cnb_log2, nE = g.cni_log2;
    const int64_t cnb_mask = ((int64_t)1 << nB) - 1, cni_mask = ((int64_t)1 << nE) - 1;
    const int G = nE < 7 ? (BM >> nE) : 1;   // rows of the tile per environment index
    constexpr int64_t PS = brick_ps(TNSLQ_BF16X3);
#pragma unroll
    for (int q = 0; q < 3; ++q) {
#pragma unroll
        for (int a = 0; a < TM; ++a) {
            const int il0 = wm * TM * 16 + a * 16;   // 32-row group (il0 >> 5) is uniform
            char *s0 = sbase(il0 >> 5), *s1 = sbase(4 + (il0 >> 5));
#pragma unroll
            for (int b = 0; b < TN; ++b)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int il = il0 + 4 * fk + r, jl = wn * TN * 16 + b * 16 + frow;
                    const float re = accr[a][b][r], im = acci[a][b][r];
                    uint16_t h[2];
                    split_bf16<2>(q == 0 ? re : (q == 1 ? im : re + im), h);
                    const int off = (il & 31) * SROW + 2 * jl;
                    *(uint16_t *)(s0 + off) = h[0];
                    *(uint16_t *)(s1 + off) = h[1];
                }
        }
        __syncthreads();
#pragma unroll
        for (int x = 0; x < 4; ++x) {
            const int R = tid + NT * x, ii = R >> 4;
            const int il = (ii % G) * (BM / G) + ii / G, jl = 8 * (R & 15);
            const int64_t i = tl.i0 + il, j = tl.j0 + jl;
            if (i < g.M && j < g.N) {
                const int64_t row = (j >> nB) * g.crs + (i >> nE);
                const int64_t col = ((i & cni_mask) << nB) + (j & cnb_mask);
                const int64_t idx = brick_index(TNSLQ_BF16X3, g.c_nst, row, col);
                const int off = (il & 31) * SROW + 2 * jl;
#pragma unroll
                for (int p = 0; p < 2; ++p)
                    *(uint4 *)((uint16_t *)g.C + idx + (2 * q + p) * PS) = *(const uint4 *)(sbase(4 * p + (il >> 5)) + off);
            }
        }
        __syncthreads();
    }
}

hipError_t launch_bf16x3(const GemmDesc &g, hipStream_t st) {
    const int64_t nblocks = ((g.M + BM - 1) / BM) * ((g.N + BN - 1) / BN) * g.S;
    if (nblocks < 1 || nblocks > 0x7fffffff) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL(k_cgemm_bf16x3, dim3((unsigned)nblocks), dim3(NT), 0, st, g);
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
        return launch_bf16x3(g, st);
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
