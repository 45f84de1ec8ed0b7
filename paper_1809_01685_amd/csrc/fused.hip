// Both contractions of the lazy partial-transpose matvec (Sec. V, Eq. 4,
// intermediary (i)) in one read of psi, for HBM-bound shapes with one vector
// and a single-qubit B (K d_B = 2).
//
// With psi regrouped as P[c][a][b] (E slowest, B fastest) each environment
// slab c is a d_A x d_B matrix M_c, and
//   Ups_c[k][b'][b] = sum_a' conj(M_c[a'][b]) X[k][a'][b']   (d_B x d_B per probe)
//   Y[k][a][b]     += sum_b' M_c[a][b'] Ups_c[k][b'][b].
// Contraction 2 of slab c needs only that slab's intermediary, so a block can
// finish one slab before the next, and the rows a thread reads in
// contraction 1 are the rows it updates in contraction 2: each thread loads
// its rows of the slab (one 16-byte unit per row; a wave's load is 1 KiB of
// consecutive rows) straight into registers, P slabs ahead in a ring, forms
// its part of Ups_c against its rows of X (held in registers for all slabs),
// the block sums the parts (wave butterflies, then the waves in order by one
// thread per entry, two barriers), and each thread adds M_c Ups_c to its rows
// of a running partial Y, also in registers.  psi is read once and the slab
// never passes through LDS.  One block per CU walks a contiguous range of
// slabs and writes its partial Y once; the Lanczos pass sums the blocks'
// partials in block order.  All products and sums are FP64, in a fixed order.
#include "tnslq_internal.h"

namespace tnslq {
namespace {

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
// thread (d_A = FT RPT), P = slabs in the ring of registers.
template <int DB, int KP, int FT, int RPT, int P>
__global__ void __launch_bounds__(FT, 1) k_pt_rows(const float4 *__restrict__ Pm, const double2 *__restrict__ X,
                                                 int64_t dE, int64_t slabs, double2 *__restrict__ Ypart) {
    static_assert(DB == 2, "rows of one 16-byte unit");
    constexpr int FW = FT / 64;                      // waves per block
    constexpr int64_t N = (int64_t)FT * RPT * DB;   // d_A d_B
    constexpr int64_t ROWS = (int64_t)FT * RPT;     // d_A: 16-byte units of a slab
    constexpr int NV = KP * DB * DB;                 // entries of one slab's intermediary
    __shared__ double red[NV][FW][2];                // each wave's part of Ups_c
    __shared__ double ups[NV][2];                    // Ups_c
    const int t = threadIdx.x, wid = t >> 6, lane = t & 63;
    const int64_t c0 = (int64_t)blockIdx.x * slabs;
    const int64_t c1 = c0 + slabs < dE ? c0 + slabs : dE;
    if (c0 >= c1) return;
    const int64_t last = c1 - 1;

    // this thread's rows a = t + r FT of the probe block, kept for every slab
    double2 x[RPT][KP][DB];
#pragma unroll
    for (int r = 0; r < RPT; ++r)
#pragma unroll
        for (int k = 0; k < KP; ++k)
#pragma unroll
            for (int bp = 0; bp < DB; ++bp) x[r][k][bp] = X[(int64_t)k * N + ((int64_t)r * FT + t) * DB + bp];
    // X complete before the slab loads start: the wait count the compiler
    // places at the loop head merges the first entry with every later one,
    // and with X's loads issued after the ring's it waits there for every
    // load in flight (vmcnt(0)), draining the ring once per P slabs
    __builtin_amdgcn_s_waitcnt(0x0f70);   // vmcnt(0)
    __builtin_amdgcn_sched_barrier(0);
    double yr[RPT][KP][DB], yi[RPT][KP][DB];
#pragma unroll
    for (int r = 0; r < RPT; ++r)
#pragma unroll
        for (int k = 0; k < KP; ++k)
#pragma unroll
            for (int b = 0; b < DB; ++b) yr[r][k][b] = yi[r][k][b] = 0.0;

    float4 ring[P][RPT];
    auto load = [&](int64_t c, float4 (&m)[RPT]) __attribute__((always_inline)) {
        const float4 *p = Pm + c * ROWS + t;
#pragma unroll
        for (int r = 0; r < RPT; ++r) m[r] = p[(int64_t)r * FT];
    };
    auto work = [&](const float4 (&m)[RPT]) __attribute__((always_inline)) {
        // this thread's part of Ups_c[k][b'][b] = sum_a conj(M[a][b]) X[k][a][b']
        double ur[KP][DB][DB], ui[KP][DB][DB];
#pragma unroll
        for (int k = 0; k < KP; ++k)
#pragma unroll
            for (int bp = 0; bp < DB; ++bp)
#pragma unroll
                for (int b = 0; b < DB; ++b) ur[k][bp][b] = ui[k][bp][b] = 0.0;
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            const double mr[DB] = {m[r].x, m[r].z}, mi[DB] = {m[r].y, m[r].w};
#pragma unroll
            for (int k = 0; k < KP; ++k)
#pragma unroll
                for (int bp = 0; bp < DB; ++bp)
#pragma unroll
                    for (int b = 0; b < DB; ++b) {
                        ur[k][bp][b] = fma(mr[b], x[r][k][bp].x, ur[k][bp][b]);
                        ur[k][bp][b] = fma(mi[b], x[r][k][bp].y, ur[k][bp][b]);
                        ui[k][bp][b] = fma(mr[b], x[r][k][bp].y, ui[k][bp][b]);
                        ui[k][bp][b] = fma(-mi[b], x[r][k][bp].x, ui[k][bp][b]);
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
                        red[v][wid][0] = sr;
                        red[v][wid][1] = si;
                    }
                }
        __syncthreads();
        if (t < NV) {
            double sr = 0.0, si = 0.0;
            for (int w = 0; w < FW; ++w) {
                sr += red[t][w][0];
                si += red[t][w][1];
            }
            ups[t][0] = sr;
            ups[t][1] = si;
        }
        __syncthreads();
        double Ur[KP][DB][DB], Ui[KP][DB][DB];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            Ur[v / (DB * DB)][(v / DB) % DB][v % DB] = ups[v][0];
            Ui[v / (DB * DB)][(v / DB) % DB][v % DB] = ups[v][1];
        }
        // Y[k][a][b] += sum_b' M[a][b'] Ups_c[k][b'][b] on this thread's rows
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            const double mr[DB] = {m[r].x, m[r].z}, mi[DB] = {m[r].y, m[r].w};
#pragma unroll
            for (int k = 0; k < KP; ++k)
#pragma unroll
                for (int b = 0; b < DB; ++b)
#pragma unroll
                    for (int bp = 0; bp < DB; ++bp) {
                        yr[r][k][b] = fma(mr[bp], Ur[k][bp][b], yr[r][k][b]);
                        yr[r][k][b] = fma(-mi[bp], Ui[k][bp][b], yr[r][k][b]);
                        yi[r][k][b] = fma(mr[bp], Ui[k][bp][b], yi[r][k][b]);
                        yi[r][k][b] = fma(mi[bp], Ur[k][bp][b], yi[r][k][b]);
                    }
        }
    };

    // slabs c0 .. c0 + P - 1 in flight, then each slab worked on and its
    // registers refilled with the slab P further on (the last slab again
    // past the end of the range, an L2 hit).  The compiler waits for every
    // load in flight at the head of a loop whose iterations use registers
    // loaded by the one before, so one iteration walks the ring UNR times:
    // that drain comes once per UNR P slabs, and within an iteration each
    // slab waits for its own loads only.  The refills are unconditional (a
    // refill inside the tail test would make every head wait as well).
    constexpr int UNR = 4;
#pragma unroll
    for (int i = 0; i < P; ++i) load(c0 + i <= last ? c0 + i : last, ring[i]);
    for (int64_t c = c0; c < c1; c += P * UNR) {
#pragma unroll
        for (int u = 0; u < UNR; ++u)
#pragma unroll
            for (int i = 0; i < P; ++i) {
                const int64_t cc = c + u * P + i;
                if (cc < c1) work(ring[i]);
                load(cc + P <= last ? cc + P : last, ring[i]);
            }
    }
    double2 *out = Ypart + (int64_t)blockIdx.x * KP * N;
#pragma unroll
    for (int r = 0; r < RPT; ++r)
#pragma unroll
        for (int k = 0; k < KP; ++k)
#pragma unroll
            for (int b = 0; b < DB; ++b)
                out[(int64_t)k * N + (t + (int64_t)r * FT) * DB + b] = make_double2(yr[r][k][b], yi[r][k][b]);
}

template <int DB, int KP, int FT, int RPT, int P>
hipError_t launch_rows(const float2 *Pm, const double2 *X, int64_t dE, int nblk, double2 *Ypart, hipStream_t st) {
    const int64_t slabs = (dE + nblk - 1) / nblk;
    hipLaunchKernelGGL((k_pt_rows<DB, KP, FT, RPT, P>), dim3(nblk), dim3(FT), 0, st, (const float4 *)Pm, X, dE,
                       slabs, Ypart);
    return hipGetLastError();
}

// Whether an instance serves (d_A, d_B, K): the shapes where one read beat
// the two streaming passes on the 30-qubit state.  d_A = 2^12 (512 threads,
// 8 rows each, 2 slabs in flight: 252 VGPRs) and 2^11 (256 threads, 8 rows,
// 3 slabs) keep X, the partial Y and the ring in registers without spilling;
// at d_A = 2^13 they would need twice the registers, and with K d_B = 4 the
// intermediary's sums and the partial Y double, so those shapes keep the two
// passes.
bool instance(int64_t dA, int64_t dB, int K) { return dB == 2 && K == 1 && (dA == 2048 || dA == 4096); }

}  // namespace

bool pt_fused_supported(int dtype, int64_t dA, int64_t dB, int K, int64_t dE) {
    return dtype == TNSLQ_C64 && dE >= 1 && instance(dA, dB, K);
}

hipError_t launch_pt_fused(const void *P, const double2 *X, int64_t dA, int64_t dB, int K, int64_t dE, int nblk,
                           double2 *Ypart, hipStream_t st) {
    if (nblk < 1 || nblk > dE) return hipErrorInvalidValue;
    const float2 *p = (const float2 *)P;
    if (!instance(dA, dB, K)) return hipErrorInvalidValue;
    if (dA == 2048) return launch_rows<2, 1, 256, 8, 3>(p, X, dE, nblk, Ypart, st);
    return launch_rows<2, 1, 512, 8, 2>(p, X, dE, nblk, Ypart, st);
}

}  // namespace tnslq
