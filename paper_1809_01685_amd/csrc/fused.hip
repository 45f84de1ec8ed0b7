// Both contractions of the lazy partial-transpose matvec (Sec. V, Eq. 4,
// intermediary (i)) in one read of psi, for HBM-bound shapes with one vector
// and a single-qubit B (K d_B = 2) and slabs of 32 or 64 KiB.
//
// With psi regrouped as P[c][a][b] (E slowest, B fastest) each environment
// slab c is a d_A x d_B matrix M_c, and
//   Ups_c[k][b'][b] = sum_a' conj(M_c[a'][b]) X[k][a'][b']   (d_B x d_B per probe)
//   Y[k][a][b]     += sum_b' M_c[a][b'] Ups_c[k][b'][b].
// Contraction 2 of slab c needs only that slab's intermediary, so one block
// can finish a slab before the next: it copies the slab from HBM into LDS
// (direct global-to-LDS loads), each thread forms its part of Ups_c over its
// rows of the slab, the block sums the parts (wave butterflies, then the
// waves in order), and each thread adds M_c Ups_c to its rows of a running
// partial Y that stays in registers for all of the block's slabs.  The slab
// is read from LDS twice and from HBM once; the probe block X (K d_A d_B
// FP64 values, the same for every slab) is read from L2 once and kept in
// registers.  The LDS holds two slab buffers: the next slab's copy is issued
// as soon as the current one has landed, so it overlaps the work on the
// current one.  One block per CU walks a contiguous range of slabs and
// writes its partial Y once; the Lanczos pass sums the blocks' partials in
// block order.  All products and sums are FP64, in a fixed order.
#include "tnslq_internal.h"

namespace tnslq {
namespace {

constexpr int SLAB_MAX = 128 * 1024;       // LDS bytes of one staged slab

typedef __attribute__((address_space(3))) void lds_void;
typedef __attribute__((address_space(1))) const void gbl_void;
typedef double d2v __attribute__((ext_vector_type(2)));
typedef float f4v __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) const d2v gd2v;
typedef __attribute__((address_space(3))) const f4v lf4v;

// v plus its DPP-moved copy (both 32-bit halves moved alike); lanes of rows
// outside ROWS add 0
template <int CTRL, int ROWS>
__device__ inline double dpp_add(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, ROWS, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROWS, 0xf, false);
    return v + __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// The sum over the wave's 64 lanes, returned to every lane: pairs, quads,
// half rows and rows of 16 by lane permutations within a row, then rows 0-1
// into row 1 and rows 0-3 into row 3 by row broadcasts; lane 63 holds the
// total.  A fixed order, done in registers.
__device__ inline double wave_total(double v) {
    v = dpp_add<0xB1, 0xf>(v);    // quad_perm [1, 0, 3, 2]
    v = dpp_add<0x4E, 0xf>(v);    // quad_perm [2, 3, 0, 1]
    v = dpp_add<0x141, 0xf>(v);   // row_half_mirror
    v = dpp_add<0x140, 0xf>(v);   // row_mirror
    v = dpp_add<0x142, 0xa>(v);   // row_bcast:15 into rows 1 and 3
    v = dpp_add<0x143, 0xc>(v);   // row_bcast:31 into rows 2 and 3
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, 63), hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// DB = d_B, KP = probes, FT = threads per block, RPT = rows of each slab per
// thread (d_A = FT RPT).
template <int DB, int KP, int FT, int RPT>
__global__ void __launch_bounds__(FT, 1) k_pt_fused(const float2 *__restrict__ P, const double2 *__restrict__ X,
                                                   int64_t dE, int64_t slabs, double2 *__restrict__ Ypart) {
    constexpr int FW = FT / 64;                      // waves per block
    constexpr int64_t N = (int64_t)FT * RPT * DB;   // d_A d_B
    constexpr int UPT = (int)(N * 8 / 16 / FT);      // 16-byte units of a slab per thread
    constexpr int NV = KP * DB * DB;                 // entries of one slab's intermediary
    // Slabs of at most 64 KiB take two LDS buffers: the next slab's copy is
    // issued as soon as the current one has landed.  That needs the
    // thread's share of X (K x RPT x DB FP64 values, at most 32 registers)
    // held in registers across slabs, since a load of X would wait for the
    // copy issued before it.  Otherwise one buffer, refilled once the slab
    // has been used, and X read again (from L2) for every slab.
    constexpr bool DOUBLE = N * 8 <= SLAB_MAX / 2 && RPT * KP * DB <= (FT <= 256 ? 32 : 8);
    constexpr bool XREG = DOUBLE;
    constexpr int UNROLL = XREG ? RPT : (DB == 4 ? 1 : 2);
    static_assert(N * 8 <= SLAB_MAX && UPT * FT * 16 == N * 8, "slab staging");
    extern __shared__ __attribute__((aligned(16))) char lds[];
    double *red = (double *)(lds + SLAB_MAX);        // [NV][FW][2]: each wave's part of Ups_c
    double *ups = red + NV * FW * 2;                 // [NV][2]: Ups_c
    const int t = threadIdx.x, wid = t >> 6, lane = t & 63;
    const int64_t c0 = (int64_t)blockIdx.x * slabs;
    const int64_t c1 = c0 + slabs < dE ? c0 + slabs : dE;

    // thread t copies units t + i FT of the slab (16 bytes each): each wave's
    // load fills 1 KiB of LDS at the same offset as in memory
    // (a block-uniform base per load plus one per-thread offset, so that
    // the addresses take scalar registers)
    const uint32_t toff = 16u * (uint32_t)t;
    auto buf = [&](int64_t c) __attribute__((always_inline)) -> uint32_t {
        return DOUBLE ? (uint32_t)((c - c0) & 1) * (SLAB_MAX / 2) : 0u;
    };
    auto fetch = [&](int64_t c) __attribute__((always_inline)) {
        const char *g = (const char *)(P + c * N) + toff;
        char *l = lds + buf(c) + 1024 * wid;
#pragma unroll 1
        for (int i = 0; i < UPT; ++i, g += FT * 16, l += FT * 16)
            __builtin_amdgcn_global_load_lds((gbl_void *)g, (lds_void *)l, 16, 0, 0);
    };
    // row a = t + r FT of the staged slab, from an LDS base the compiler
    // must take as given, so that the second read of a row is a read and not
    // a copy kept in registers from the first
    static_assert(DB % 2 == 0, "rows of whole 16-byte units");
    auto load_row = [&](int r, uint32_t base, float2 *m) __attribute__((always_inline)) {
        lf4v *p = (lf4v *)(uintptr_t)(base + (uint32_t)(t + r * FT) * (DB * 8u));
#pragma unroll
        for (int i = 0; i < DB / 2; ++i) {
            const f4v v = p[i];
            m[2 * i] = make_float2(v.x, v.y);
            m[2 * i + 1] = make_float2(v.z, v.w);
        }
    };

    double yr[RPT][KP][DB], yi[RPT][KP][DB];
#pragma unroll
    for (int r = 0; r < RPT; ++r)
#pragma unroll
        for (int k = 0; k < KP; ++k)
#pragma unroll
            for (int b = 0; b < DB; ++b) yr[r][k][b] = yi[r][k][b] = 0.0;

    if (c0 < c1) fetch(c0);
    for (int64_t c = c0; c < c1; ++c) {
        __builtin_amdgcn_s_waitcnt(0x0f70);   // vmcnt(0): this wave's part of slab c has landed
        __syncthreads();                      // (and every thread is done with slab c - 1)
        if constexpr (DOUBLE)
            if (c + 1 < c1) fetch(c + 1);     // into the buffer slab c - 1 used
        // without XREG the compiler must not keep X's loads across slabs
        uint64_t xaddr = (uint64_t)X;
        if constexpr (!XREG) asm volatile("" : "+s"(xaddr));
        const gd2v *Xc = (const gd2v *)xaddr;
        const uint32_t lbase = (uint32_t)(uintptr_t)(__attribute__((address_space(3))) char *)lds + buf(c);

        // this thread's part of Ups_c: ur/ui[k][b'][b] = sum_r conj(M[a_r][b]) X[k][a_r][b']
        double ur[KP][DB][DB], ui[KP][DB][DB];
#pragma unroll
        for (int k = 0; k < KP; ++k)
#pragma unroll
            for (int bp = 0; bp < DB; ++bp)
#pragma unroll
                for (int b = 0; b < DB; ++b) ur[k][bp][b] = ui[k][bp][b] = 0.0;
        // (a rolled loop: only the running partial Y needs its rows unrolled
        // into registers, and a rolled loop keeps few rows' loads in flight)
#pragma unroll UNROLL
        for (int r = 0; r < RPT; ++r) {
            float2 m[DB];
            load_row(r, lbase, m);
#pragma unroll
            for (int k = 0; k < KP; ++k) {
                // X[k][a][.] for a = t + r FT: uniform base, per-thread offset t DB
                const gd2v *xr = (const gd2v *)((const __attribute__((address_space(1))) char *)(
                                                    Xc + (int64_t)k * N + (int64_t)r * FT * DB) +
                                                (uint32_t)t * (DB * 16u));
                double2 x[DB];
#pragma unroll
                for (int bp = 0; bp < DB; ++bp) {
                    const d2v v = xr[bp];
                    x[bp] = make_double2(v.x, v.y);
                }
#pragma unroll
                for (int bp = 0; bp < DB; ++bp)
#pragma unroll
                    for (int b = 0; b < DB; ++b) {
                        // conj(M[a'][b]) x[b']
                        const double mr = m[b].x, mi = m[b].y;
                        ur[k][bp][b] = fma(mr, x[bp].x, ur[k][bp][b]);
                        ur[k][bp][b] = fma(mi, x[bp].y, ur[k][bp][b]);
                        ui[k][bp][b] = fma(mr, x[bp].y, ui[k][bp][b]);
                        ui[k][bp][b] = fma(-mi, x[bp].x, ui[k][bp][b]);
                    }
            }
        }
        // the block's sum: each wave's in registers, then the waves' parts in
        // order by one thread per entry
#pragma unroll
        for (int k = 0; k < KP; ++k)
#pragma unroll
            for (int bp = 0; bp < DB; ++bp)
#pragma unroll
                for (int b = 0; b < DB; ++b) {
                    const int v = (k * DB + bp) * DB + b;
                    const double sr = wave_total(ur[k][bp][b]), si = wave_total(ui[k][bp][b]);
                    if (lane == 0) {
                        red[(v * FW + wid) * 2] = sr;
                        red[(v * FW + wid) * 2 + 1] = si;
                    }
                }
        __syncthreads();
        if (t < NV) {
            double sr = 0.0, si = 0.0;
            for (int w = 0; w < FW; ++w) {
                sr += red[(t * FW + w) * 2];
                si += red[(t * FW + w) * 2 + 1];
            }
            ups[2 * t] = sr;
            ups[2 * t + 1] = si;
        }
        __syncthreads();
        double Ur[KP][DB][DB], Ui[KP][DB][DB];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            Ur[v / (DB * DB)][(v / DB) % DB][v % DB] = ups[2 * v];
            Ui[v / (DB * DB)][(v / DB) % DB][v % DB] = ups[2 * v + 1];
        }
        // Y[k][a][b] += sum_b' M[a][b'] Ups[k][b'][b] on this thread's rows
        uint32_t ubase = lbase;
        asm volatile("" : "+v"(ubase));
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            float2 m[DB];
            load_row(r, ubase, m);
#pragma unroll
            for (int k = 0; k < KP; ++k)
#pragma unroll
                for (int b = 0; b < DB; ++b)
#pragma unroll
                    for (int bp = 0; bp < DB; ++bp) {
                        const double mr = m[bp].x, mi = m[bp].y;
                        yr[r][k][b] = fma(mr, Ur[k][bp][b], yr[r][k][b]);
                        yr[r][k][b] = fma(-mi, Ui[k][bp][b], yr[r][k][b]);
                        yi[r][k][b] = fma(mr, Ui[k][bp][b], yi[r][k][b]);
                        yi[r][k][b] = fma(mi, Ur[k][bp][b], yi[r][k][b]);
                    }
        }
        if constexpr (!DOUBLE) {
            __syncthreads();                  // every row used: the buffer takes the next slab
            if (c + 1 < c1) fetch(c + 1);
        }
    }
    // the block's partial Y[k][a][b]
    double2 *out = Ypart + (int64_t)blockIdx.x * KP * N;
#pragma unroll
    for (int r = 0; r < RPT; ++r)
#pragma unroll
        for (int k = 0; k < KP; ++k)
#pragma unroll
            for (int b = 0; b < DB; ++b)
                out[(int64_t)k * N + (t + (int64_t)r * FT) * DB + b] = make_double2(yr[r][k][b], yi[r][k][b]);
}

template <int DB, int KP, int FT, int RPT>
hipError_t launch_one(const float2 *P, const double2 *X, int64_t dE, int nblk, double2 *Ypart, hipStream_t st) {
    constexpr size_t LDS = SLAB_MAX + (size_t)(FT / 64 + 1) * KP * DB * DB * 16;
    static bool attr_set = false;
    if (!attr_set) {
        const hipError_t e = hipFuncSetAttribute((const void *)k_pt_fused<DB, KP, FT, RPT>,
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)LDS);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    const int64_t slabs = (dE + nblk - 1) / nblk;
    hipLaunchKernelGGL((k_pt_fused<DB, KP, FT, RPT>), dim3(nblk), dim3(FT), LDS, st, P, X, dE, slabs, Ypart);
    return hipGetLastError();
}

// Whether an instance serves (d_A, d_B, K): the shapes where one read beat
// the two streaming passes on the 30-qubit state (d_B = 2, K = 1, d_A = 2^11
// and 2^12: 1.3-1.4x per matvec).  With smaller slabs the per-slab sums and barriers
// dominate, with K d_B = 4 the intermediary's sums and the registers of the
// running partial Y, and at d_A = 2^13 one 128 KiB slab fills the LDS, so the
// next slab's copy cannot overlap the work on the current one; those shapes
// keep the two passes.
bool instance(int64_t dA, int64_t dB, int K) { return dB == 2 && K == 1 && (dA == 2048 || dA == 4096); }

}  // namespace

bool pt_fused_supported(int dtype, int64_t dA, int64_t dB, int K, int64_t dE) {
    return dtype == TNSLQ_C64 && dE >= 1 && instance(dA, dB, K) && dA * dB * 8 <= SLAB_MAX;
}

hipError_t launch_pt_fused(const void *P, const double2 *X, int64_t dA, int64_t dB, int K, int64_t dE, int nblk,
                           double2 *Ypart, hipStream_t st) {
    if (nblk < 1 || nblk > dE) return hipErrorInvalidValue;
    const float2 *p = (const float2 *)P;
    if (!instance(dA, dB, K)) return hipErrorInvalidValue;
    // 2048 rows: four waves with eight rows each (fewer waves in the per-slab
    // sums); 4096 rows: sixteen waves with four rows each
    if (dA == 2048) return launch_one<2, 1, 256, 8>(p, X, dE, nblk, Ypart, st);
    return launch_one<2, 1, 1024, 4>(p, X, dE, nblk, Ypart, st);
}

}  // namespace tnslq
