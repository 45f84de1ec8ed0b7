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
#include <type_traits>

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

// The same regrouping through LDS tiles, for D >= 2^TB: a tile is the 2^TB
// elements that share every output bit outside td.wr.  They are read with the
// input's lowest bits varying fastest (td.rd lists the tile's output bits in
// that order: a wave reads runs of consecutive psi elements) and written with
// the output's lowest bits varying fastest (td.wr: runs of consecutive panel
// elements).  One LDS row of padding per 64 entries keeps the transposed
// accesses off a single bank.
struct RegroupTile {
    int nouter;
    int outer[TNSLQ_MAX_QUBITS];   // output bits outside the tile, from the tile index
    int rd[12], wr[12];            // the tile's output bits in read and in write order
    int rd2wr[12];                 // position of rd[k] in wr
    int64_t in_rd[12];             // psi index bit of rd[k]
};

template <int DTYPE, int TB>
__global__ void __launch_bounds__(256) k_regroup_tiled(const void *__restrict__ psi, void *__restrict__ out,
                                                       int64_t R, int64_t C, int cl, PermDesc pd, RegroupTile td) {
    using T = typename std::conditional<DTYPE == TNSLQ_C128, double2, float2>::type;
    constexpr int TN = 1 << TB;
    __shared__ T tile[TN + TN / 64];
    const int64_t ntiles = (R * C) >> TB;
    const int wl = cl < 9 ? cl : 9;
    for (int64_t tl = blockIdx.x; tl < ntiles; tl += gridDim.x) {
        int64_t ob = 0;
        for (int k = 0; k < td.nouter; ++k) ob |= ((tl >> k) & 1) << td.outer[k];
        int64_t ib = 0;
        for (int t = 0; t < pd.L; ++t) ib |= ((ob >> t) & 1) << pd.map[t];
        for (int j = threadIdx.x; j < TN; j += 256) {
            int64_t in = ib;
            int slot = 0;
#pragma unroll
            for (int k = 0; k < TB; ++k) {
                const int bit = (j >> k) & 1;
                in |= (int64_t)bit << td.in_rd[k];
                slot |= bit << td.rd2wr[k];
            }
            tile[slot + (slot >> 6)] = ((const T *)psi)[in];
        }
        __syncthreads();
        for (int j = threadIdx.x; j < TN; j += 256) {
            int64_t o = ob;
#pragma unroll
            for (int k = 0; k < TB; ++k) o |= (int64_t)((j >> k) & 1) << td.wr[k];
            // panel_index with R, C, and the panel width min(C, 512) powers of two
            const int64_t i = o >> cl, c = o & (C - 1);
            const int64_t dst = ((c >> wl) * R << wl) + (i << wl) + (c & ((int64_t(1) << wl) - 1));
            ((T *)out)[dst] = tile[j + (j >> 6)];
        }
        __syncthreads();
    }
}

// The two adjacent elements (i, c), (i, c + 1) at panel offset e of M, read
// as a stream (nontemporal: psi is not re-read within a pass).
template <int DTYPE>
__device__ inline void load_pair(const void *M, int64_t e, double2 &a, double2 &b) {
    typedef __attribute__((ext_vector_type(4))) float f4;
    typedef __attribute__((ext_vector_type(2))) double d2;
    if constexpr (DTYPE == TNSLQ_C128) {
        const d2 x = __builtin_nontemporal_load((const d2 *)M + e);
        const d2 y = __builtin_nontemporal_load((const d2 *)M + e + 1);
        a = make_double2(x.x, x.y);
        b = make_double2(y.x, y.y);
    } else {
        const f4 f = __builtin_nontemporal_load((const f4 *)((const float2 *)M + e));
        a = make_double2(f.x, f.y);
        b = make_double2(f.z, f.w);
    }
}

// out(s, v, c) = sum over rows i of split s of op(M[i][c]) V(v, i) for the KG
// vectors v = blockIdx.z KG ..; op = conj if CONJ; M in panel layout.  A block
// covers one panel: its threads take column pairs (2 cp, 2 cp + 1), and when
// the panel is narrower than 512 columns the threads left over walk
// interleaved rows (phase ph of nph) and their sums meet in LDS at the end.
// The vector entries of a chunk of rows are staged in LDS and broadcast, each
// read serving two columns.
template <int DTYPE, bool CONJ, int KG, bool WIDE>
__global__ void __launch_bounds__(CM_THREADS) k_colmac(ColmacDesc g) {
    constexpr int U = 8;                      // rows whose loads are issued together
    constexpr int CM_CH = WIDE ? 64 : 256;    // rows of vector entries staged per chunk
    __shared__ double2 vs[KG][CM_CH];
    __shared__ double2 red[WIDE ? 1 : CM_THREADS][CM_CPT];
    const int t = threadIdx.x;
    // WIDE: the panel is 512 columns wide, one row phase
    const int64_t w = WIDE ? CM_COLS : g.C;
    const int cpairs = WIDE ? CM_THREADS : (int)(w / CM_CPT), nph = WIDE ? 1 : CM_THREADS / cpairs;
    const int cp = WIDE ? t : t % cpairs, ph = WIDE ? 0 : t / cpairs;
    const int64_t c = (int64_t)blockIdx.x * CM_COLS + CM_CPT * cp;
    const int s = blockIdx.y;
    const int v0 = blockIdx.z * KG;
    const int kn = g.NV - v0 < KG ? g.NV - v0 : KG;
    const int64_t i0 = (int64_t)s * g.rows_per_split;
    const int64_t i1 = i0 + g.rows_per_split < g.R ? i0 + g.rows_per_split : g.R;
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
            double2 v = make_double2(0.0, 0.0);
            if (k < kn && ii < nrow) {
                const int64_t vv = v0 + k;
                v = g.V[(vv >> g.vsh) * g.vs1 + (vv & ((1 << g.vsh) - 1)) * g.vs2 + (ib + ii) * g.vsi];
            }
            vs[k][ii] = v;
        }
        __syncthreads();
        if (c < g.C) {
            const int64_t base = panel_index(ib, c, g.R, g.C);
            for (int u0 = ph; u0 < nrow; u0 += U * nph) {
                // the U row loads of a batch are issued before any is used
                double2 ma[U], mb[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int ii = u0 + u * nph;
                    if (ii < nrow) {
                        load_pair<DTYPE>(g.M, base + (int64_t)ii * w, ma[u], mb[u]);
                    } else {
                        ma[u] = make_double2(0.0, 0.0);
                        mb[u] = ma[u];
                    }
                }
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int ii = u0 + u * nph;
                    const double ax = ma[u].x, ay = CONJ ? -ma[u].y : ma[u].y;
                    const double bx = mb[u].x, by = CONJ ? -mb[u].y : mb[u].y;
#pragma unroll
                    for (int k = 0; k < KG; ++k) {
                        // rows past the chunk load zeros; any staged entry will do
                        const double2 v = vs[k][ii < CM_CH ? ii : 0];
                        ar[0][k] = fma(ax, v.x, fma(-ay, v.y, ar[0][k]));
                        ai[0][k] = fma(ax, v.y, fma(ay, v.x, ai[0][k]));
                        ar[1][k] = fma(bx, v.x, fma(-by, v.y, ar[1][k]));
                        ai[1][k] = fma(bx, v.y, fma(by, v.x, ai[1][k]));
                    }
                }
            }
        }
    }
    // phases of one column pair add up (one vector at a time through LDS)
#pragma unroll
    for (int k = 0; k < KG; ++k) {
        double2 r0 = make_double2(ar[0][k], ai[0][k]), r1 = make_double2(ar[1][k], ai[1][k]);
        if (!WIDE && nph > 1) {
            __syncthreads();
            red[t][0] = r0;
            red[t][1] = r1;
            __syncthreads();
            if (ph == 0) {
                for (int p = 1; p < nph; ++p) {
                    const double2 x0 = red[p * cpairs + cp][0], x1 = red[p * cpairs + cp][1];
                    r0.x += x0.x;
                    r0.y += x0.y;
                    r1.x += x1.x;
                    r1.y += x1.y;
                }
            }
        }
        if (ph == 0 && c < g.C && k < kn) {
            const int64_t vv = v0 + k;
            double2 *o = g.out + s * g.osplit + (vv >> g.osh) * g.os1 + (vv & ((1 << g.osh) - 1)) * g.os2;
            o[c * g.osc] = r0;
            o[(c + 1) * g.osc] = r1;
        }
    }
}

// The plain case of the column MAC: full 512-column panels, vectors
// V[v][i] = V[v R + i] and output out[s][v][c] (the entropy's two passes).
// The same sums with simpler addressing, which keeps the kernel at 4 waves
// per SIMD with 8 vectors.
template <int DTYPE, bool CONJ, int KG>
__global__ void __launch_bounds__(CM_THREADS) k_colmac_plain(ColmacDesc g) {
    constexpr int U = 8, CH = 64;
    __shared__ double2 vs[KG][CH];
    const int t = threadIdx.x;
    const int64_t c = ((int64_t)blockIdx.x * CM_THREADS + t) * CM_CPT;
    const int s = blockIdx.y;
    const int v0 = blockIdx.z * KG;
    const int kn = g.NV - v0 < KG ? g.NV - v0 : KG;
    const int64_t i0 = (int64_t)s * g.rows_per_split;
    const int64_t i1 = i0 + g.rows_per_split < g.R ? i0 + g.rows_per_split : g.R;
    double ar[CM_CPT][KG], ai[CM_CPT][KG];
#pragma unroll
    for (int j = 0; j < CM_CPT; ++j)
#pragma unroll
        for (int k = 0; k < KG; ++k) ar[j][k] = ai[j][k] = 0.0;
    for (int64_t ib = i0; ib < i1; ib += CH) {
        const int nrow = (int)(i1 - ib < CH ? i1 - ib : CH);
        __syncthreads();
        for (int e = t; e < KG * CH; e += CM_THREADS) {
            const int k = e / CH, ii = e % CH;
            vs[k][ii] = (k < kn && ii < nrow) ? g.V[(int64_t)(v0 + k) * g.R + ib + ii] : make_double2(0.0, 0.0);
        }
        __syncthreads();
        const int64_t base = panel_index(ib, c, g.R, g.C);
        for (int u0 = 0; u0 < nrow; u0 += U) {
            double2 ma[U], mb[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (u0 + u < nrow) {
                    load_pair<DTYPE>(g.M, base + (int64_t)(u0 + u) * CM_COLS, ma[u], mb[u]);
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
                    const double2 v = vs[k][(u0 + u) & (CH - 1)];
                    ar[0][k] = fma(ax, v.x, fma(-ay, v.y, ar[0][k]));
                    ai[0][k] = fma(ax, v.y, fma(ay, v.x, ai[0][k]));
                    ar[1][k] = fma(bx, v.x, fma(-by, v.y, ar[1][k]));
                    ai[1][k] = fma(bx, v.y, fma(by, v.x, ai[1][k]));
                }
            }
        }
    }
#pragma unroll
    for (int k = 0; k < KG; ++k)
        if (k < kn) {
            double2 *o = g.out + s * g.osplit + (int64_t)(v0 + k) * g.C + c;
            o[0] = make_double2(ar[0][k], ai[0][k]);
            o[1] = make_double2(ar[1][k], ai[1][k]);
        }
}

// The plain column MAC for groups of 8 (NVG = 1) or 16 (NVG = 2) vectors on
// the FP64 matrix instructions (full 512-column panels, rows per split a
// multiple of 4).  Per 4 rows, each 16-column tile of M takes per group of 8
// vectors two v_mfma_f64_16x16x4f64 into one accumulator:
//   D = Mr [Vr | Vi] + Mi [-Vi | Vr]        (M V)
//   D = Mr [Vr | Vi] + Mi [Vi | -Vr]        (conj(M) V)
// (16 x 4 blocks of M's real and imaginary parts against 4 x 16 blocks of the
// eight vectors' real and imaginary parts), so that D's column j < 8 is the
// real and j >= 8 the imaginary part of vector j % 8.  A wave owns NQ runs of
// 32 columns, each the even and the odd columns' tiles (NQ = 2 / NVG: 32
// accumulator registers, four waves per SIMD; a block covers 128 NQ columns
// of a panel).  Lane l loads the column pair 2 (l % 16), 2 (l % 16) + 1 of a
// run in row l / 16 of the 4 (the A operand: row l % 16 of a tile, term
// l / 16), reads vector entry (l % 8, row l / 16) of each group from LDS (the
// B operand: term l / 16, column l % 16), and holds D's rows 4 r + l / 16,
// column l % 16, in register r.
template <int DTYPE, bool CONJ, int NVG>
__global__ void __launch_bounds__(CM_THREADS) k_colmac_mfma(ColmacDesc g) {
    typedef __attribute__((ext_vector_type(4))) double f64x4;
    constexpr int KG = 8 * NVG, CH = 64;        // vectors per group, vector rows staged per chunk
    constexpr int NQ = 2 / NVG;                 // 32-column runs per wave
    constexpr int BPP = CM_COLS / (128 * NQ);   // blocks per panel
    __shared__ double2 vs[KG][CH];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int fr = lane & 15, fk = lane >> 4;
    const int s = blockIdx.y;
    const int v0 = blockIdx.z * KG;
    const int kn = g.NV - v0 < KG ? g.NV - v0 : KG;
    const int64_t i0 = (int64_t)s * g.rows_per_split;
    const int64_t i1 = i0 + g.rows_per_split;
    const int64_t pc0 = (int64_t)(blockIdx.x % BPP) * 128 * NQ + (int64_t)w * 32 * NQ + 2 * fr;
    const int64_t pbase = (int64_t)(blockIdx.x / BPP) * g.R * CM_COLS;   // the panel
    f64x4 acc[NQ][2][NVG];
#pragma unroll
    for (int q = 0; q < NQ; ++q)
#pragma unroll
        for (int h = 0; h < NVG; ++h) acc[q][0][h] = acc[q][1][h] = f64x4{0.0, 0.0, 0.0, 0.0};
    const int vj = fr & 7;
    const bool imag_col = fr >= 8;
    for (int64_t ib = i0; ib < i1; ib += CH) {
        const int nrow = (int)(i1 - ib < CH ? i1 - ib : CH);
        __syncthreads();
        for (int e = t; e < KG * CH; e += CM_THREADS) {
            const int k = e / CH, ii = e % CH;
            vs[k][ii] = (k < kn && ii < nrow) ? g.V[(int64_t)(v0 + k) * g.R + ib + ii] : make_double2(0.0, 0.0);
        }
        __syncthreads();
        for (int r0 = 0; r0 < nrow; r0 += 4) {
            const int rr = r0 + fk;   // this lane's row of the step
            double2 ma[NQ], mb[NQ];
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                if (rr < nrow) {
                    load_pair<DTYPE>(g.M, pbase + (ib + rr) * CM_COLS + pc0 + 32 * q, ma[q], mb[q]);
                } else {
                    ma[q] = make_double2(0.0, 0.0);
                    mb[q] = ma[q];
                }
            }
#pragma unroll
            for (int h = 0; h < NVG; ++h) {
                const double2 v = vs[8 * h + vj][rr < CH ? rr : 0];
                const double bp = imag_col ? v.y : v.x;
                const double bq = CONJ ? (imag_col ? -v.x : v.y) : (imag_col ? v.x : -v.y);
#pragma unroll
                for (int q = 0; q < NQ; ++q) {
                    acc[q][0][h] = __builtin_amdgcn_mfma_f64_16x16x4f64(ma[q].x, bp, acc[q][0][h], 0, 0, 0);
                    acc[q][0][h] = __builtin_amdgcn_mfma_f64_16x16x4f64(ma[q].y, bq, acc[q][0][h], 0, 0, 0);
                    acc[q][1][h] = __builtin_amdgcn_mfma_f64_16x16x4f64(mb[q].x, bp, acc[q][1][h], 0, 0, 0);
                    acc[q][1][h] = __builtin_amdgcn_mfma_f64_16x16x4f64(mb[q].y, bq, acc[q][1][h], 0, 0, 0);
                }
            }
        }
    }
    // D row 4 r + fk of tile (q, e) is column 128 NQ blockIdx.x + 32 NQ w + 32 q + 2 (4 r + fk) + e
    const int64_t cb = (int64_t)blockIdx.x * 128 * NQ + (int64_t)w * 32 * NQ;
#pragma unroll
    for (int h = 0; h < NVG; ++h) {
        if (8 * h + vj >= kn) continue;
        double *o = (double *)(g.out + s * g.osplit + (int64_t)(v0 + 8 * h + vj) * g.C) + (imag_col ? 1 : 0);
#pragma unroll
        for (int q = 0; q < NQ; ++q)
#pragma unroll
            for (int e = 0; e < 2; ++e)
#pragma unroll
                for (int r = 0; r < 4; ++r) o[2 * (cb + 32 * q + 2 * (4 * r + fk) + e)] = acc[q][e][h][r];
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

// The streaming form of the partial-transpose matvec: the first pass leaves
// Up[s][(k, b')][(c, b)] (split partials over a'); the second pass wants
// U2[(k, b)][(c, b')] as its vectors over the reduction index (c, b').
__global__ void __launch_bounds__(256) k_sum_transpose_ups(const double2 *__restrict__ Up, int S, int64_t n, int nB,
                                                           int nE, double2 *__restrict__ U2) {
    const int64_t dB = int64_t(1) << nB, dE = int64_t(1) << nE;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) {
        // e = ((k dB + b) dE + c) dB + b'
        const int64_t bp = e & (dB - 1), c = (e >> nB) & (dE - 1), b = (e >> (nB + nE)) & (dB - 1);
        const int64_t k = e >> (2 * nB + nE);
        const int64_t src = ((k << nB) + bp) * (dE * dB) + (c << nB) + b;
        double x = 0.0, y = 0.0;
        for (int p = 0; p < S; ++p) {
            const double2 v = Up[p * n + src];
            x += v.x;
            y += v.y;
        }
        U2[e] = make_double2(x, y);
    }
}

// The streaming partial-transpose matvec's first pass takes its vectors over
// a': Lanczos vectors xq[k][a dB + b] -> Xq[(k, b)][a], K dA dB elements.
__global__ void __launch_bounds__(256) k_vectors_by_b(const double2 *__restrict__ xq, int64_t total, int64_t dA,
                                                      int nB, double2 *__restrict__ Xq) {
    const int64_t dB = int64_t(1) << nB, n = dA * dB;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
        const int64_t a = e % dA, kb = e / dA;
        Xq[e] = xq[(kb >> nB) * n + a * dB + (kb & (dB - 1))];
    }
}

// Its second pass leaves Yt[s][(k, b)][a]; Y[k][a dB + b] = sum_s Yt[s].
__global__ void __launch_bounds__(256) k_sum_transpose_y(const double2 *__restrict__ Yt, int S, int64_t total,
                                                         int64_t dA, int nB, double2 *__restrict__ Y) {
    const int64_t dB = int64_t(1) << nB, n = dA * dB;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
        const int64_t k = e / n, r = e % n;
        const int64_t src = ((k << nB) + (r & (dB - 1))) * dA + (r >> nB);
        double x = 0.0, y = 0.0;
        for (int p = 0; p < S; ++p) {
            const double2 v = Yt[p * total + src];
            x += v.x;
            y += v.y;
        }
        Y[e] = make_double2(x, y);
    }
}

}  // namespace

hipError_t launch_vectors_by_b(const double2 *xq, int K, int64_t dA, int nB, double2 *Xq, hipStream_t st) {
    const int64_t total = (int64_t)K * dA * (int64_t(1) << nB);
    int64_t g = (total + 255) / 256;
    if (g > 8192) g = 8192;
    hipLaunchKernelGGL(k_vectors_by_b, dim3((unsigned)g), dim3(256), 0, st, xq, total, dA, nB, Xq);
    return hipGetLastError();
}

hipError_t launch_sum_transpose_y(const double2 *Yt, int S, int K, int64_t dA, int nB, double2 *Y, hipStream_t st) {
    const int64_t total = (int64_t)K * dA * (int64_t(1) << nB);
    int64_t g = (total + 255) / 256;
    if (g > 8192) g = 8192;
    hipLaunchKernelGGL(k_sum_transpose_y, dim3((unsigned)g), dim3(256), 0, st, Yt, S, total, dA, nB, Y);
    return hipGetLastError();
}

hipError_t launch_regroup(int dtype, const void *psi, void *out, int64_t R, int64_t C, const PermDesc &pd,
                          hipStream_t st) {
    const int TB = dtype == TNSLQ_C128 ? 11 : 12;   // 33 KiB of LDS either way
    if (pd.L >= TB) {
        // the tile: the output's 6 lowest bits, the output bits of psi's
        // lowest TB - 6 bits, then further output bits up to TB
        RegroupTile td{};
        int inv[TNSLQ_MAX_QUBITS];
        for (int t = 0; t < pd.L; ++t) inv[pd.map[t]] = t;
        int in_tile[TNSLQ_MAX_QUBITS] = {0};
        int nu = 0, u[12];
        auto add = [&](int b) {
            if (nu < TB && !in_tile[b]) {
                in_tile[b] = 1;
                u[nu++] = b;
            }
        };
        for (int b = 0; b < 6; ++b) add(b);
        for (int b = 0; b < TB - 6; ++b) add(inv[b]);
        for (int b = 6; b < pd.L && nu < TB; ++b) add(b);
        // write order: ascending output bits; read order: psi's lowest bits first
        int nw = 0, nr = 0;
        for (int b = 0; b < pd.L; ++b)
            if (in_tile[b]) td.wr[nw++] = b;
        int used[TNSLQ_MAX_QUBITS] = {0};
        for (int b = 0; b < pd.L && nr < TB; ++b) {
            const int ob = inv[b];
            if (in_tile[ob] && !used[ob]) {
                used[ob] = 1;
                td.rd[nr++] = ob;
            }
        }
        for (int k = 0; k < TB; ++k) {
            for (int w = 0; w < TB; ++w)
                if (td.wr[w] == td.rd[k]) td.rd2wr[k] = w;
            td.in_rd[k] = pd.map[td.rd[k]];
        }
        td.nouter = 0;
        for (int b = 0; b < pd.L; ++b)
            if (!in_tile[b]) td.outer[td.nouter++] = b;
        int cl = 0;
        while ((int64_t(1) << cl) < C) ++cl;
        const int64_t ntiles = (R * C) >> TB;
        const unsigned g = (unsigned)(ntiles < 65535 * 8 ? ntiles : 65535 * 8);
        if (dtype == TNSLQ_C128)
            hipLaunchKernelGGL((k_regroup_tiled<TNSLQ_C128, 11>), dim3(g), dim3(256), 0, st, psi, out, R, C, cl, pd, td);
        else
            hipLaunchKernelGGL((k_regroup_tiled<TNSLQ_C64, 12>), dim3(g), dim3(256), 0, st, psi, out, R, C, cl, pd, td);
        return hipGetLastError();
    }
    int64_t g = (R * C + 1023) / 1024;
    if (g < 1) g = 1;
    if (g > 65535 * 8) g = 65535 * 8;
    if (dtype == TNSLQ_C128)
        hipLaunchKernelGGL((k_regroup<TNSLQ_C128>), dim3((unsigned)g), dim3(256), 0, st, psi, out, R, C, pd);
    else
        hipLaunchKernelGGL((k_regroup<TNSLQ_C64>), dim3((unsigned)g), dim3(256), 0, st, psi, out, R, C, pd);
    return hipGetLastError();
}

template <int KG, bool WIDE>
void colmac_kg(int dtype, int conj, dim3 grid, hipStream_t st, const ColmacDesc &g) {
    const bool plain = WIDE && g.vsh == 0 && g.vs1 == g.R && g.vsi == 1 && g.osh == 0 && g.os1 == g.C && g.osc == 1;
#define TNSLQ_CM(T, CJ)                                                                                   \
    do {                                                                                                  \
        if (plain)                                                                                        \
            hipLaunchKernelGGL((k_colmac_plain<T, CJ, KG>), grid, dim3(CM_THREADS), 0, st, g);           \
        else                                                                                              \
            hipLaunchKernelGGL((k_colmac<T, CJ, KG, WIDE>), grid, dim3(CM_THREADS), 0, st, g);           \
    } while (0)
    if (dtype == TNSLQ_C128) {
        if (conj) TNSLQ_CM(TNSLQ_C128, true);
        else TNSLQ_CM(TNSLQ_C128, false);
    } else {
        if (conj) TNSLQ_CM(TNSLQ_C64, true);
        else TNSLQ_CM(TNSLQ_C64, false);
    }
#undef TNSLQ_CM
}

hipError_t launch_colmac(int dtype, int conj, ColmacDesc g, hipStream_t st) {
    if (g.R < 1 || g.C < CM_CPT || g.NV < 1 || g.S < 1 || g.R % g.S != 0 || g.C % CM_CPT != 0) return hipErrorInvalidValue;
    if (g.C < CM_COLS && CM_COLS % g.C != 0) return hipErrorInvalidValue;   // narrow panels: C divides 512
    if (g.vsh < 0 || g.vsh > 30 || g.osh < 0 || g.osh > 30) return hipErrorInvalidValue;
    g.rows_per_split = g.R / g.S;
    // more than 4 vectors over full panels in 4-row steps: the matrix
    // instructions, 8 or 16 vectors per pass over M (16 and several passes
    // beyond)
    const bool plain = g.vsh == 0 && g.vs1 == g.R && g.vsi == 1 && g.osh == 0 && g.os1 == g.C && g.osc == 1;
    if (g.NV > 4 && plain && g.C % CM_COLS == 0 && g.rows_per_split % 4 == 0) {
        const int nvg = g.NV > 8 ? 2 : 1;
        const int64_t gx = (g.C / CM_COLS) * (nvg == 1 ? 2 : 4), gz = (g.NV + 8 * nvg - 1) / (8 * nvg);
        if (gx > 0x7fffffff || g.S > 65535 || gz > 65535) return hipErrorInvalidConfiguration;
        const dim3 grid((unsigned)gx, (unsigned)g.S, (unsigned)gz);
#define TNSLQ_CMM(T, CJ, G) hipLaunchKernelGGL((k_colmac_mfma<T, CJ, G>), grid, dim3(CM_THREADS), 0, st, g)
        if (dtype == TNSLQ_C128) {
            if (conj) {
                if (nvg == 1) TNSLQ_CMM(TNSLQ_C128, true, 1);
                else TNSLQ_CMM(TNSLQ_C128, true, 2);
            } else {
                if (nvg == 1) TNSLQ_CMM(TNSLQ_C128, false, 1);
                else TNSLQ_CMM(TNSLQ_C128, false, 2);
            }
        } else {
            if (conj) {
                if (nvg == 1) TNSLQ_CMM(TNSLQ_C64, true, 1);
                else TNSLQ_CMM(TNSLQ_C64, true, 2);
            } else {
                if (nvg == 1) TNSLQ_CMM(TNSLQ_C64, false, 1);
                else TNSLQ_CMM(TNSLQ_C64, false, 2);
            }
        }
#undef TNSLQ_CMM
        return hipGetLastError();
    }
    // vectors per pass over M: the smallest of 1, 2, 4, 8 covering NV (8 and
    // several passes beyond)
    const int kg = g.NV <= 1 ? 1 : g.NV <= 2 ? 2 : g.NV <= 4 ? 4 : 8;
    const int64_t gx = (g.C + CM_COLS - 1) / CM_COLS, gz = (g.NV + kg - 1) / kg;
    if (gx > 0x7fffffff || g.S > 65535 || gz > 65535) return hipErrorInvalidConfiguration;
    const dim3 grid((unsigned)gx, (unsigned)g.S, (unsigned)gz);
    // full panels (C a multiple of 512) compile without the row phases
    const bool wide = g.C >= CM_COLS;
    switch (kg) {
        case 1: wide ? colmac_kg<1, true>(dtype, conj, grid, st, g) : colmac_kg<1, false>(dtype, conj, grid, st, g); break;
        case 2: wide ? colmac_kg<2, true>(dtype, conj, grid, st, g) : colmac_kg<2, false>(dtype, conj, grid, st, g); break;
        case 4: wide ? colmac_kg<4, true>(dtype, conj, grid, st, g) : colmac_kg<4, false>(dtype, conj, grid, st, g); break;
        default: wide ? colmac_kg<8, true>(dtype, conj, grid, st, g) : colmac_kg<8, false>(dtype, conj, grid, st, g); break;
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

hipError_t launch_sum_transpose_ups(const double2 *Up, int S, int K, int nB, int nE, double2 *U2, hipStream_t st) {
    const int64_t n = (int64_t)K << (2 * nB + nE);
    int64_t g = (n + 255) / 256;
    if (g > 65535 * 4) g = 65535 * 4;
    if (g < 1) g = 1;
    hipLaunchKernelGGL(k_sum_transpose_ups, dim3((unsigned)g), dim3(256), 0, st, Up, S, n, nB, nE, U2);
    return hipGetLastError();
}

}  // namespace tnslq
