// C ABI and host orchestration of libtnslq.
//
// The host side validates arguments, plans the layout and the workspace
// carve-up, and drives the device loop of Algorithm 1 (Sec. III): one block
// matvec (both contractions of Sec. V Eq. 4) per Lanczos step for all probes
// at once, the FP64 recurrence, and at the end the Gauss quadrature and the
// Hutchinson statistics.  No device memory is allocated here.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <mutex>
#include <string>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "tnslq_internal.h"

using namespace tnslq;

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define TNSLQ_HIP(x)                                                                          \
    do {                                                                                      \
        hipError_t e_ = (x);                                                                  \
        if (e_ != hipSuccess) return fail(TNSLQ_E_DEVICE, "%s: %s", #x, hipGetErrorString(e_)); \
    } while (0)

constexpr size_t ALIGN = 256;
inline size_t up(size_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }

// Largest intermediary (Ups) chunk the planner allows, in complex values
// (16 GiB in FP32, 24 GiB in split BF16, 32 GiB in FP64 bricks).
constexpr size_t UPS_BUDGET_VALUES = size_t(1) << 31;
// Blocks per probe vector of the Lanczos kernels' two-stage reductions: at
// least 4096 elements per block for long vectors, but enough blocks over the
// K probes to fill the chip (about 2048) down to 128 elements per block.
int reduction_blocks(int64_t n, int K) {
    const int64_t want = std::max<int64_t>(n / 4096, (2048 + K - 1) / K);
    const int64_t cap = std::min<int64_t>(1024, std::max<int64_t>(1, n / 128));
    return (int)std::max<int64_t>(1, std::min(want, cap));
}

// Largest explicit operator (intermediary (iii)): d_A d_B, and bytes of the
// operator and of its dense FP32/FP64 precursor.
constexpr int64_t EXPLICIT_MAX_N = 16384;
constexpr size_t EXPLICIT_BUDGET = size_t(4) << 30;
// the streaming form of the lazy operator up to this many vectors K d_B (up
// to 4 its passes run on the vector units, up to 8 on the FP64 matrix
// instructions, both at the HBM rate; from 16 the split-BF16 bricks are faster)
constexpr int64_t STREAM_MAX_VECTORS = 8;
// intermediates of the factorised MPS operator (probes are chunked to fit)
constexpr size_t MPS_BUDGET = size_t(8) << 30;

int check_partition(const tnslq_partition *p) {
    if (!p) return fail(TNSLQ_E_ARG, "partition is NULL");
    if (p->n_qubits < 1 || p->n_qubits > TNSLQ_MAX_QUBITS)
        return fail(TNSLQ_E_PARTITION, "n_qubits %d outside [1, %d]", p->n_qubits, TNSLQ_MAX_QUBITS);
    if (p->n_a < 0 || p->n_b < 0 || p->n_a + p->n_b > p->n_qubits)
        return fail(TNSLQ_E_PARTITION, "bad subsystem sizes n_a=%d n_b=%d", p->n_a, p->n_b);
    if ((p->n_a > 0 && !p->a) || (p->n_b > 0 && !p->b)) return fail(TNSLQ_E_ARG, "qubit list is NULL");
    std::vector<int> seen(p->n_qubits, 0);
    for (int i = 0; i < p->n_a + p->n_b; ++i) {
        const int q = i < p->n_a ? p->a[i] : p->b[i - p->n_a];
        if (q < 0 || q >= p->n_qubits) return fail(TNSLQ_E_PARTITION, "qubit %d out of range", q);
        if (seen[q]) return fail(TNSLQ_E_PARTITION, "qubit %d listed twice", q);
        seen[q] = 1;
    }
    return TNSLQ_OK;
}

int check_prec(int prec) {
    if (prec < TNSLQ_FP64 || prec > TNSLQ_BF16X6) return fail(TNSLQ_E_ARG, "precision %d unknown", prec);
    return TNSLQ_OK;
}
int check_dtype(int dtype) {
    if (dtype != TNSLQ_C64 && dtype != TNSLQ_C128) return fail(TNSLQ_E_DTYPE, "dtype %d unknown", dtype);
    return TNSLQ_OK;
}

inline int64_t up128(int64_t x) { return (x + 127) / 128 * 128; }
int plan_rest(Plan &pl, int dtype, int prec, int K, int lanczos);

// Padded complex multiply-adds of one lazy block matvec (both contractions
// over all probe chunks; matrix-core tiles are 128 x 128) and of the explicit
// form (forming rho^{T_B} once, then one dense product per matvec), for the
// operator-form choice.
double lazy_macs(const Plan &pl) {
    const int64_t chunks = (pl.K + pl.kc - 1) / pl.kc, N = up128((int64_t)pl.kc * pl.dB);
    return (double)chunks * ((double)up128(pl.dB * pl.dE) * N * pl.dA + (double)up128(pl.dA) * N * pl.dE * pl.dB);
}
double explicit_macs(int64_t n, int64_t dE, int K, int m) {
    return (double)up128(n) * up128(n) * dE + (double)m * up128(n) * up128(K) * n;
}
size_t explicit_bytes(int prec, int64_t n) {
    return std::max(brick_bytes(prec, n, n), (size_t)(n * n) * (prec == TNSLQ_FP64 ? 16 : 8));
}

// Build the plan: the operator form (Sec. V: the subsystem sizes decide
// between the lazy intermediaries and the explicit operator), roles (for the
// lazy form A and B are exchanged when B is larger, so that the contraction
// cost D * min(d_A, d_B) per probe is the smaller one), chunking and the
// workspace carve-up.  `lanczos` = 0 plans a bare lazy matvec.
int make_plan(int dtype, const tnslq_partition *p, int K, int m, int reorth, int prec, int lanczos, int opform,
              Plan &pl, int chunk = 0) {
    int rc;
    if ((rc = check_dtype(dtype)) || (rc = check_partition(p)) || (rc = check_prec(prec))) return rc;
    if (opform < TNSLQ_OPERATOR_AUTO || opform > TNSLQ_OPERATOR_LAZY_TWO_PASS)
        return fail(TNSLQ_E_ARG, "operator_form %d unknown", opform);
    if (K < 1 || K > 65535) return fail(TNSLQ_E_ARG, "n_probes %d outside [1, 65535]", K);
    if (lanczos && (m < 1 || m > TNSLQ_MAX_STEPS))
        return fail(TNSLQ_E_ARG, "n_steps %d outside [1, %d]", m, TNSLQ_MAX_STEPS);
    pl = Plan();
    pl.kc_cap = std::max(0, chunk);
    pl.two_pass = opform == TNSLQ_OPERATOR_LAZY_TWO_PASS;
    pl.L = p->n_qubits;
    pl.dtype = dtype;
    pl.prec = prec;
    pl.K = K;
    pl.m = lanczos ? m : 1;
    pl.reorth = lanczos ? (reorth ? 1 : 0) : 0;
    pl.swapped = p->n_b > p->n_a;
    // the explicit form keeps the caller's roles
    {
        const int64_t n0 = int64_t(1) << (p->n_a + p->n_b);
        const int64_t dE0 = int64_t(1) << (p->n_qubits - p->n_a - p->n_b);
        const bool fits = n0 <= EXPLICIT_MAX_N && explicit_bytes(prec, n0) <= EXPLICIT_BUDGET;
        if (lanczos && opform == TNSLQ_OPERATOR_EXPLICIT) {
            if (!fits)
                return fail(TNSLQ_E_ARG, "explicit operator: d_A d_B = %lld exceeds %lld", (long long)n0,
                            (long long)EXPLICIT_MAX_N);
            pl.expl = 1;
        } else if (lanczos && opform == TNSLQ_OPERATOR_AUTO && fits) {
            // cost of the lazy plan (roles as above, chunking as below)
            Plan lz;
            if ((rc = make_plan(dtype, p, K, m, reorth, prec, lanczos, TNSLQ_OPERATOR_LAZY, lz, chunk))) return rc;
            if (!lz.stream && explicit_macs(n0, dE0, K, lz.m) < lz.m * lazy_macs(lz)) pl.expl = 1;
        }
        if (pl.expl) pl.swapped = 0;
    }
    const int *qa = pl.swapped ? p->b : p->a;
    const int *qb = pl.swapped ? p->a : p->b;
    pl.nA = pl.swapped ? p->n_b : p->n_a;
    pl.nB = pl.swapped ? p->n_a : p->n_b;
    for (int i = 0; i < pl.nA; ++i) pl.qa[i] = qa[i];
    for (int i = 0; i < pl.nB; ++i) pl.qb[i] = qb[i];
    std::vector<int> used(pl.L, 0);
    for (int i = 0; i < p->n_a; ++i) used[p->a[i]] = 1;
    for (int i = 0; i < p->n_b; ++i) used[p->b[i]] = 1;
    pl.nE = 0;
    for (int q = 0; q < pl.L; ++q)
        if (!used[q]) pl.qe[pl.nE++] = q;
    pl.dA = int64_t(1) << pl.nA;
    pl.dB = int64_t(1) << pl.nB;
    pl.dE = int64_t(1) << pl.nE;
    pl.dAB = pl.dA * pl.dB;
    pl.D = int64_t(1) << pl.L;
    return plan_rest(pl, dtype, prec, K, lanczos);
}

// The network form's tensors (offsets from pl.off_net): E_W regrouped
// [(m, n')][(m', n)] (a gap), E_Z regrouped [(u, v')][(v, u')] (a ring),
// their complex64 copies, and four scratch tensors of up to s4 entries for
// the normalisation (Gram matrices of the blocks, E_W, E_Z and their
// contractions, each at most (bond^2)^2).
struct NetBufs {
    size_t ewp, ezp, ew32, ez32, x[4], total;
    int64_t s4;
};
NetBufs net_bufs(const Plan &pl) {
    NetBufs b{};
    const int64_t UM = pl.nU * pl.nM, NV = pl.nN * pl.nV, MN = pl.nM * pl.nN, UV = pl.nU * pl.nV,
                  UN = pl.nU * pl.nN;
    const int64_t w = std::max({UM, NV, MN, UV, UN});
    b.s4 = w * w;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t r = o;
        o += up(std::max<size_t>(bytes, 16));
        return r;
    };
    b.ewp = take(pl.ngap ? (size_t)MN * MN * 16 : 16);
    b.ezp = take(pl.nring ? (size_t)UV * UV * 16 : 16);
    const bool f32 = pl.prec == TNSLQ_FP32;
    b.ew32 = take(pl.ngap && f32 ? (size_t)MN * MN * 8 : 16);
    b.ez32 = take(pl.nring && f32 ? (size_t)UV * UV * 8 : 16);
    for (int i = 0; i < 4; ++i) b.x[i] = take((size_t)b.s4 * 16);
    b.total = o;
    return b;
}

// Chunking, splits and the workspace carve-up of a plan whose roles, sizes
// and operator form are set.
int plan_rest(Plan &pl, int dtype, int prec, int K, int lanczos) {
    const size_t acc = prec == TNSLQ_FP64 ? 16 : 8;
    pl.nst1 = brick_stages(prec, pl.dA);
    pl.nst2 = brick_stages(prec, pl.dE * pl.dB);
    // intermediary per probe: d_B rows (b) by d_E d_B reduction terms (c, b')
    const size_t ups_values_per = (size_t)brick_rows(pl.dB) * brick_stages(prec, pl.dE * pl.dB) * brick_epr(prec);
    pl.kc = (int)std::max<int64_t>(
        1, std::min<int64_t>(K, (int64_t)(UPS_BUDGET_VALUES / std::max<size_t>(ups_values_per, 1))));
    if (pl.kc_cap > 0) pl.kc = std::min(pl.kc, pl.kc_cap);
    // every chunk must start on a block of 128 rows (k, b') of Xt (lazy form:
    // d_B is then a power of two, so below 128 it divides 128; the factorised
    // MPS operator chunks its probes on its own, below)
    if (!pl.expl && !pl.mpsf && pl.kc < K && (pl.kc * pl.dB) % BRICK_ROWS != 0) {
        const int q = (int)(BRICK_ROWS / pl.dB);
        pl.kc = std::min(K, (pl.kc + q - 1) / q * q);
    }
    // split-K of the second contraction: enough blocks to fill the chip,
    // at least 8 bricks per split
    const int64_t tiles = ((pl.dA + 127) / 128) * ((pl.kc * pl.dB + 127) / 128);
    pl.S = 1;
    while (tiles * pl.S < 2048 && pl.nst2 % (2 * pl.S) == 0 && pl.nst2 / (2 * pl.S) >= 8) pl.S *= 2;
    // the first contraction too, when its output (d_B d_E x kc d_B) has few
    // tiles: partial sums in the accumulator type, merged into Ups afterwards
    const int64_t tiles1 = ((pl.dB * pl.dE + 127) / 128) * ((pl.kc * pl.dB + 127) / 128);
    pl.S1 = 1;
    if (tiles1 < 1024)
        while (tiles1 * pl.S1 < 2048 && pl.nst1 % (2 * pl.S1) == 0 && pl.nst1 / (2 * pl.S1) >= 8) pl.S1 *= 2;
    const int64_t n = pl.dAB;
    pl.nblk = reduction_blocks(n, K);
    // HBM regime: with K d_B <= STREAM_MAX_VECTORS vectors the contractions do
    // at most that many complex multiply-adds per element of psi and the
    // 128 x 128 matrix-core tiles would be mostly padding; they run instead as
    // two streaming passes over psi in its own dtype with FP64 products and sums.
    pl.stream = !pl.expl && !pl.mpsf && (int64_t)K * pl.dB <= STREAM_MAX_VECTORS;
    if (pl.expl) {
        // one dense product per matvec: rho^{T_B} (n rows, reduction n) with
        // the K vectors (rows k, reduction n), split-K to fill the chip
        pl.kc = K;
        pl.S1 = 1;
        pl.nst1 = pl.nst_rho = brick_stages(prec, n);
        pl.nst_e = brick_stages(prec, pl.dE);
        const int64_t tl = (up128(n) / 128) * (up128(K) / 128);
        pl.S = 1;
        while (tl * pl.S < 2048 && pl.nst_rho % (2 * pl.S) == 0 && pl.nst_rho / (2 * pl.S) >= 8) pl.S *= 2;
    }
    if (pl.stream) {
        pl.kc = K;
        pl.S1 = 1;
        // pass 1: d_A rows, d_E d_B columns (one block per 512); pass 2: d_E d_B
        // rows, d_A columns
        const int64_t gx1 = (pl.dE * pl.dB + 511) / 512, gx2 = (pl.dA + 511) / 512;
        pl.S1s = 1;
        while (gx1 * pl.S1s < 2048 && pl.dA / (2 * pl.S1s) >= 256) pl.S1s *= 2;
        pl.S2s = 1;
        while (gx2 * pl.S2s < 2048 && pl.dE * pl.dB / (2 * pl.S2s) >= 64) pl.S2s *= 2;
        pl.S = pl.S2s;
        // one read of psi where the shape has an instance and every CU gets a
        // slab range (fused.hip)
        pl.fused = !pl.two_pass && pl.dE >= FUSED_BLOCKS && pt_fused_supported(dtype, pl.dA, pl.dB, K, pl.dE);
        if (pl.fused) pl.S = FUSED_BLOCKS;
    }

    // factorised MPS operator: four complex products per probe, chunks of
    // probes within a fixed budget of intermediates
    // (network form: Z1 = T1, Z2 and Z2p = T2 .. T4, Z3 = T5, with U'M -> U M
    // and MV -> N V)
    const int64_t UpM = pl.mnet ? pl.nU * pl.nM : pl.mUp * pl.mM, MV = pl.mnet ? pl.nN * pl.nV : pl.mM * pl.mV;
    const size_t mes = prec == TNSLQ_FP32 ? 8 : 16;   // bytes per complex entry of its intermediates
    if (pl.mpsf) {
        const size_t per = mes * (size_t)(UpM * pl.dB + 2 * UpM * MV + pl.dA * MV + 2 * n);
        pl.kc = (int)std::max<int64_t>(1, std::min<int64_t>({(int64_t)K, (int64_t)(MPS_BUDGET / per), 65535}));
        pl.S1 = 1;
        // the last product (d_A' x d_B' outputs, a sum over MV terms) has few
        // output tiles: split its reduction until the chunk fills the chip,
        // at least 256 terms per split; passA sums the splits
        const int64_t ytiles = ((pl.dA + 63) / 64) * ((pl.dB + 63) / 64) * pl.kc;
        pl.S = 1;
        while (ytiles * pl.S < 1024 && MV / (2 * pl.S) >= 256 && (int64_t)pl.kc * 2 * pl.S <= 65535) pl.S *= 2;
    }

    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t r = o;
        o += up(bytes);
        return r;
    };
    if (pl.mpsf) {
        pl.off_mps = take(pl.mps_bytes);
        pl.off_Z1 = take((size_t)pl.kc * UpM * pl.dB * mes);
        pl.off_Z2 = take((size_t)pl.kc * UpM * MV * mes);
        pl.off_Z2p = take((size_t)pl.kc * UpM * MV * mes);
        pl.off_Z3 = take((size_t)pl.kc * pl.dA * MV * mes);
        pl.off_Ypart = take((size_t)pl.S * pl.kc * n * mes);
        pl.off_nrm = take(pl.mnet ? 64 : (size_t)2 * pl.mM * pl.mM * 16 + 64);
        if (pl.mnet) pl.off_net = take(net_bufs(pl).total);
        if (prec == TNSLQ_FP32) {
            pl.off_P32 = take((size_t)pl.dA * UpM * 8);     // P or R_A
            pl.off_Q32 = take((size_t)pl.dB * MV * 8);      // Q or R_B
            pl.off_X32 = take((size_t)pl.kc * n * 8);
        }
    } else if (pl.expl) {
        pl.off_Pabe = take(brick_bytes(prec, n, pl.dE));
        pl.off_Pabc = take(brick_bytes(prec, n, pl.dE));
        pl.off_Cd = take((size_t)(n * n) * acc);
        pl.off_rho = take(brick_bytes(prec, n, n));
        pl.off_Xt = take(brick_bytes(prec, K, n));
        pl.off_Ypart = take((size_t)pl.S * K * n * acc);
    } else if (pl.stream && pl.fused) {
        pl.off_P1s = take((size_t)8 * pl.D);                        // psi as P[c][a][b]
        pl.off_Ypart = take((size_t)FUSED_BLOCKS * K * n * 16);     // the blocks' partial Y
        if (!lanczos) pl.off_Xs = take((size_t)K * n * 16);
    } else if (pl.stream) {
        const size_t esz = dtype == TNSLQ_C128 ? 16 : 8;
        const int64_t nv = (int64_t)K * pl.dB, ncol = pl.dE * pl.dB;
        pl.off_P1s = take(esz * (size_t)pl.D);
        pl.off_P2s = take(esz * (size_t)pl.D);
        pl.off_Up = take((size_t)pl.S1s * nv * ncol * 16);
        pl.off_U2 = take((size_t)nv * ncol * 16);
        pl.off_Ypart = take((size_t)pl.S2s * K * n * 16);
        pl.off_Xq = take((size_t)K * n * 16);
        pl.off_Ym = take((size_t)K * n * 16);
        if (!lanczos) pl.off_Xs = take((size_t)K * n * 16);
    } else {
        pl.off_Paeb = take(brick_bytes(prec, pl.dA, pl.dE * pl.dB));
        pl.off_Pbea = take(brick_bytes(prec, pl.dB * pl.dE, pl.dA));
        pl.off_Xt = take(brick_bytes(prec, (int64_t)K * pl.dB, pl.dA));
        pl.off_Ups = take(brick_bytes(prec, (int64_t)pl.kc * pl.dB, pl.dE * pl.dB));
        pl.off_Ypart = take((size_t)pl.S * pl.kc * n * acc);
        if (pl.S1 > 1) pl.off_U1part = take((size_t)pl.S1 * pl.kc * pl.dB * pl.dE * pl.dB * acc);
    }
    if (lanczos) {
        pl.nQ = pl.reorth ? pl.m + 1 : 3;
        pl.off_Q = take((size_t)pl.nQ * K * n * 16);
        pl.off_w = take((size_t)K * n * 16);
        pl.off_alpha = take((size_t)K * pl.m * 8);
        pl.off_beta = take((size_t)K * (pl.m + 1) * 8);
        pl.off_F = take((size_t)K * pl.m * 8);
        pl.off_G = take((size_t)K * 8);
        pl.off_stats = take((size_t)pl.m * 4 * 8);
        pl.off_red = take((size_t)2 * K * pl.nblk * 8);
        pl.off_h = take((size_t)K * (pl.m + 1) * pl.nblk * 16 + (size_t)K * (pl.m + 1) * 16);
        pl.off_steps = take((size_t)K * 4);
        pl.off_fit = take((size_t)2 * K * 8 + 8 * 8);
        pl.off_feat = take(64 * 4);
        pl.off_mlp = take(mlp_ws_bytes(1) + 64);
        pl.off_chk = take(STATE_CHECK_BYTES);
    }
    pl.total = o;
    return TNSLQ_OK;
}

// Sites of general local dimension (explicit form only): A and B in the
// order given, E the other sites in increasing order; psi's flat index in
// mixed radix with site 0 most significant.
int check_partition_dims(const tnslq_partition_dims *p) {
    if (!p) return fail(TNSLQ_E_ARG, "partition is NULL");
    if (p->n_sites < 1 || p->n_sites > TNSLQ_MAX_QUBITS)
        return fail(TNSLQ_E_PARTITION, "n_sites %d outside [1, %d]", p->n_sites, TNSLQ_MAX_QUBITS);
    if (!p->dims) return fail(TNSLQ_E_ARG, "dims is NULL");
    if (p->n_a < 0 || p->n_b < 0 || p->n_a + p->n_b > p->n_sites)
        return fail(TNSLQ_E_PARTITION, "bad subsystem sizes n_a=%d n_b=%d", p->n_a, p->n_b);
    if ((p->n_a > 0 && !p->a) || (p->n_b > 0 && !p->b)) return fail(TNSLQ_E_ARG, "site list is NULL");
    int64_t D = 1;
    for (int s = 0; s < p->n_sites; ++s) {
        if (p->dims[s] < 2 || p->dims[s] > 65536)
            return fail(TNSLQ_E_PARTITION, "site %d: dimension %d outside [2, 65536]", s, p->dims[s]);
        if (D > (int64_t(1) << 40) / p->dims[s]) return fail(TNSLQ_E_PARTITION, "state dimension exceeds 2^40");
        D *= p->dims[s];
    }
    std::vector<int> seen(p->n_sites, 0);
    for (int i = 0; i < p->n_a + p->n_b; ++i) {
        const int q = i < p->n_a ? p->a[i] : p->b[i - p->n_a];
        if (q < 0 || q >= p->n_sites) return fail(TNSLQ_E_PARTITION, "site %d out of range", q);
        if (seen[q]) return fail(TNSLQ_E_PARTITION, "site %d listed twice", q);
        seen[q] = 1;
    }
    return TNSLQ_OK;
}

int make_plan_dims(int dtype, const tnslq_partition_dims *p, int K, int m, int reorth, int prec, int lanczos,
                   int opform, Plan &pl) {
    int rc;
    if ((rc = check_dtype(dtype)) || (rc = check_prec(prec)) || (rc = check_partition_dims(p))) return rc;
    int64_t D = 1;
    for (int s = 0; s < p->n_sites; ++s) D *= p->dims[s];
    std::vector<int> seen(p->n_sites, 0);
    for (int i = 0; i < p->n_a; ++i) seen[p->a[i]] = 1;
    for (int i = 0; i < p->n_b; ++i) seen[p->b[i]] = 1;
    if (K < 1 || K > 65535) return fail(TNSLQ_E_ARG, "n_probes %d outside [1, 65535]", K);
    if (lanczos && (m < 1 || m > TNSLQ_MAX_STEPS))
        return fail(TNSLQ_E_ARG, "n_steps %d outside [1, %d]", m, TNSLQ_MAX_STEPS);
    if (opform == TNSLQ_OPERATOR_LAZY || opform == TNSLQ_OPERATOR_LAZY_TWO_PASS)
        return fail(TNSLQ_E_ARG, "sites of general dimension take the explicit operator only");
    if (opform < TNSLQ_OPERATOR_AUTO || opform > TNSLQ_OPERATOR_EXPLICIT)
        return fail(TNSLQ_E_ARG, "operator_form %d unknown", opform);
    pl = Plan();
    pl.L = p->n_sites;
    pl.dtype = dtype;
    pl.prec = prec;
    pl.K = K;
    pl.m = lanczos ? m : 1;
    pl.reorth = lanczos ? (reorth ? 1 : 0) : 0;
    pl.expl = 1;
    pl.mixed = 1;
    std::vector<int64_t> stride(p->n_sites);
    int64_t acc = 1;
    for (int s = p->n_sites - 1; s >= 0; --s) {
        stride[s] = acc;
        acc *= p->dims[s];
    }
    std::vector<int> grp[3];
    grp[0].assign(p->a, p->a + p->n_a);
    grp[1].assign(p->b, p->b + p->n_b);
    for (int s = 0; s < p->n_sites; ++s)
        if (!seen[s]) grp[2].push_back(s);
    for (int g = 0; g < 3; ++g) {
        pl.md.n[g] = (int)grp[g].size();
        pl.md.d[g] = 1;
        for (int i = 0; i < pl.md.n[g]; ++i) {
            pl.md.dim[g][i] = p->dims[grp[g][i]];
            pl.md.stride[g][i] = stride[grp[g][i]];
            pl.md.d[g] *= p->dims[grp[g][i]];
        }
    }
    pl.dA = pl.md.d[0];
    pl.dB = pl.md.d[1];
    pl.dE = pl.md.d[2];
    pl.dAB = pl.dA * pl.dB;
    pl.D = D;
    if (pl.dAB > EXPLICIT_MAX_N || explicit_bytes(prec, pl.dAB) > EXPLICIT_BUDGET)
        return fail(TNSLQ_E_ARG, "explicit operator: d_A d_B = %lld exceeds %lld", (long long)pl.dAB,
                    (long long)EXPLICIT_MAX_N);
    return plan_rest(pl, dtype, prec, K, lanczos);
}

// Output bit t of the regrouped index <- input bit of psi's flat index.
// `order` lists the three groups from most to least significant.
PermDesc perm_for(const Plan &pl, const int *g0, int n0, const int *g1, int n1, const int *g2, int n2) {
    PermDesc pd{};
    pd.L = pl.L;
    int t = 0;
    const int *groups[3] = {g2, g1, g0};
    const int sizes[3] = {n2, n1, n0};
    for (int gi = 0; gi < 3; ++gi)
        for (int i = sizes[gi] - 1; i >= 0; --i) pd.map[t++] = pl.L - 1 - groups[gi][i];
    return pd;
}

// Output bit t <- input bit, for psi regrouped with group `hi` most
// significant and group `lo` least significant.
PermDesc perm_two(int L, const int *hi, int n_hi, const int *lo, int n_lo) {
    PermDesc pd{};
    pd.L = L;
    int t = 0;
    for (int i = n_lo - 1; i >= 0; --i) pd.map[t++] = L - 1 - lo[i];
    for (int i = n_hi - 1; i >= 0; --i) pd.map[t++] = L - 1 - hi[i];
    return pd;
}

// Column MAC over an R x C matrix with K plain vectors V[k][i] and output
// out[s][k][c].
ColmacDesc plain_colmac(const void *M, int64_t R, int64_t C, const double2 *V, int K, double2 *out, int S) {
    ColmacDesc g{};
    g.M = M;
    g.R = R;
    g.C = C;
    g.V = V;
    g.NV = K;
    g.vsh = 0;
    g.vs1 = R;
    g.vs2 = 0;
    g.vsi = 1;
    g.out = out;
    g.osplit = (int64_t)K * C;
    g.osh = 0;
    g.os1 = C;
    g.os2 = 0;
    g.osc = 1;
    g.S = S;
    return g;
}

// ------------------------------------------------------------ MPS blocks
int64_t ceil_pow2_log(int64_t x) {
    int q = 0;
    while ((int64_t(1) << q) < x) ++q;
    return q;
}

// Sizes and workspace of the effective state of two contiguous blocks of an
// open or periodic MPS (Sec. VI); see tnslq_mps_effective_state.
constexpr int64_t MPS_CHOL_MAX = 16384;           // widest factored matrix
constexpr int64_t MPS_EXPLICIT_AUTO = int64_t(1) << 26;   // largest explicit section the automatic choice keeps

// One section of the chain: its sites in order (consecutive along the ring),
// the bonds x entering and y leaving it, its physical size p (saturated above
// 2^40), whether it is compressed (p > x y), and if so whether its matrix
// comes from the transfer sweep (tr) or from the explicit section.
struct MpsSec {
    std::vector<int> sites;
    int64_t x = 1, y = 1, p = 1;
    bool comp = false, tr = false;
    int64_t smax = 0;             // explicit: the largest running section
    int64_t tmax = 0, amax = 0;   // transfer: the largest T and step scratch
};

struct MpsPlan {
    int L = 0, a0 = 0, a1 = 0, b0 = 0, b1 = 0;
    bool closed = false;
    std::vector<int> p, bond;
    std::vector<int64_t> off;          // element offset of each site's tensor
    MpsSec A, B, G, O;                 // blocks, gap (empty when adjacent), a ring's outer section
    int64_t U = 1, Mb = 1, Nb = 1, V = 1;
    int64_t kA = 1, kB = 1, Wd = 1, Zd = 1;
    int64_t Up = 1, Mf = 1, Vf = 1;    // psi[a][b][(u', v')] = sum_m P[a][u'][m] Q[b][m][v']
    int q[3] = {0, 0, 0};
    int64_t smax = 1, gmax = 1, maxb = 1, tmax = 1, amax = 1;
    size_t off_El[2], off_Er[2], off_S[3], off_SA, off_SB, off_SG, off_SO, off_G, off_RA, off_RB, off_RBp, off_W,
        off_Z, off_T1, off_T, off_P, off_Q2, off_Q2p, off_TT, off_Tt[2], off_At, off_part, off_fail, total = 0;
};

// Physical size, compression and route of a section: 0, or 1 when the
// explicit section the route needs would exceed 2^31 entries, 2 when the
// transfer sweep's buffers would exceed 2^32 entries.
int plan_sec(const MpsPlan &mp, MpsSec &s, int route, bool absorb_right) {
    const int64_t LIM = int64_t(1) << 40;
    s.x = mp.bond[s.sites.front()];
    s.y = mp.bond[s.sites.back() + 1];
    s.p = 1;
    for (int i : s.sites) s.p = s.p > LIM / mp.p[i] ? LIM + 1 : s.p * mp.p[i];
    s.comp = s.p > s.x * s.y;
    // explicit: running section x (physical so far) bond; transfer: x^2 bond^2
    // and the step's x^2 bond p bond (complex multiply-adds as costs)
    double ex = 0.0, tr = (double)s.x * s.x * s.x * s.x, f = 1.0;
    int64_t rows = s.x;
    bool fits = true;
    s.smax = s.amax = 0;
    s.tmax = s.x * s.x * s.x * s.x;   // the sweep's start
    for (int i : s.sites) {
        const int64_t z = mp.bond[i], y = mp.bond[(size_t)i + 1], pi = mp.p[i];
        ex += (double)rows * z * pi * y;
        f *= pi;
        if (fits && (double)rows * pi * y <= (double)(int64_t(1) << 31)) {
            rows *= pi;
            s.smax = std::max(s.smax, rows * y);
        } else {
            fits = false;
        }
        tr += (double)s.x * s.x * pi * z * y * (double)(z + y);
        s.tmax = std::max(s.tmax, s.x * s.x * y * y);
        s.amax = std::max(s.amax, s.x * s.x * z * pi * y);
    }
    if (absorb_right) {
        s.smax = std::max(s.smax, rows * s.y);
        s.amax = std::max(s.amax, s.x * s.x * s.y * s.y);
    }
    ex += (double)s.x * s.y * s.x * s.y * f;   // the Gram product over the physical index
    const bool tfits = std::max(s.tmax, s.amax) <= (int64_t(1) << 32);
    if (!s.comp)
        s.tr = false;
    else if (route == TNSLQ_MPS_SECTIONS_TRANSFER)
        s.tr = true;
    else if (route == TNSLQ_MPS_SECTIONS_EXPLICIT)
        s.tr = false;
    else
        s.tr = tfits && (!fits || s.smax > MPS_EXPLICIT_AUTO || tr < ex);
    if (s.tr) {
        s.smax = 0;
        return tfits ? 0 : 2;
    }
    s.tmax = s.amax = 0;
    return fits ? 0 : 1;
}

// dense: room for the effective state itself (the dense route); without it
// only the factors are built, or with net only the network form's pieces.
int plan_mps(const tnslq_mps *m, int a0, int na, int b0, int nb, MpsPlan &mp, bool dense = true, bool net = false) {
    if (!m) return fail(TNSLQ_E_ARG, "mps is NULL");
    const int L = m->n_sites;
    if (L < 2 || L > 100000) return fail(TNSLQ_E_ARG, "n_sites %d outside [2, 100000]", L);
    if (!m->phys || !m->bond) return fail(TNSLQ_E_ARG, "phys or bond is NULL");
    if (m->sections < TNSLQ_MPS_SECTIONS_AUTO || m->sections > TNSLQ_MPS_SECTIONS_TRANSFER)
        return fail(TNSLQ_E_ARG, "sections %d is not a TNSLQ_MPS_SECTIONS_ value", m->sections);
    if (m->bond[0] != m->bond[L])
        return fail(TNSLQ_E_ARG, "boundary bonds differ: bond[0] = %d, bond[n] = %d (open chains have 1, rings the "
                                 "same closing bond)",
                    m->bond[0], m->bond[L]);
    if (a0 < 0 || na < 1 || nb < 1 || a0 + na > b0 || b0 + nb > L)
        return fail(TNSLQ_E_PARTITION, "blocks [%d, %d) and [%d, %d) not ordered inside the chain", a0, a0 + na, b0,
                    b0 + nb);
    mp = MpsPlan();
    mp.L = L;
    mp.a0 = a0;
    mp.a1 = a0 + na;
    mp.b0 = b0;
    mp.b1 = b0 + nb;
    mp.p.assign(m->phys, m->phys + L);
    mp.bond.assign(m->bond, m->bond + L + 1);
    mp.off.resize(L + 1);
    mp.off[0] = 0;
    for (int i = 0; i <= L; ++i)
        if (mp.bond[i] < 1 || mp.bond[i] > 4096) return fail(TNSLQ_E_ARG, "bond %d: %d outside [1, 4096]", i, mp.bond[i]);
    mp.closed = mp.bond[0] > 1;
    for (int i = 0; i < L; ++i) {
        if (mp.p[i] < 2 || mp.p[i] > 65536) return fail(TNSLQ_E_ARG, "site %d: phys %d outside [2, 65536]", i, mp.p[i]);
        mp.off[i + 1] = mp.off[i] + (int64_t)mp.bond[i] * mp.p[i] * mp.bond[i + 1];
        mp.maxb = std::max<int64_t>(mp.maxb, mp.bond[i + 1]);
    }
    const bool gap = mp.b0 > mp.a1;
    for (int i = mp.a0; i < mp.a1; ++i) mp.A.sites.push_back(i);
    for (int i = mp.b0; i < mp.b1; ++i) mp.B.sites.push_back(i);
    for (int i = mp.a1; i < mp.b0; ++i) mp.G.sites.push_back(i);
    if (mp.closed) {
        for (int i = mp.b1; i < L; ++i) mp.O.sites.push_back(i);
        for (int i = 0; i < mp.a0; ++i) mp.O.sites.push_back(i);
    }
    const int route = m->sections;
    MpsSec *secs[4] = {&mp.A, &mp.B, gap ? &mp.G : nullptr, mp.O.sites.empty() ? nullptr : &mp.O};
    static const char *sname[4] = {"block A", "block B", "the gap", "the outer section"};
    int serr[4] = {0, 0, 0, 0};
    for (int k = 0; k < 4; ++k)
        if (secs[k]) serr[k] = plan_sec(mp, *secs[k], route, k == 1 && !mp.closed);
    mp.U = mp.bond[mp.a0];
    mp.Mb = mp.bond[mp.a1];
    mp.Nb = mp.bond[mp.b0];
    mp.V = mp.bond[mp.b1];
    mp.kA = mp.A.comp ? mp.U * mp.Mb : mp.A.p;
    mp.kB = mp.B.comp ? mp.Nb * mp.V : mp.B.p;
    if (gap) mp.Wd = mp.G.comp ? mp.Mb * mp.Nb : mp.G.p;
    if (mp.closed) mp.Zd = mp.O.sites.empty() ? 1 : (mp.O.comp ? mp.V * mp.U : mp.O.p);
    if (mp.closed) {
        mp.Up = gap ? mp.Wd : 1;
        mp.Mf = (gap ? mp.Nb : mp.Mb) * mp.U;
        mp.Vf = mp.Zd;
    } else {
        mp.Up = gap ? mp.U * mp.Wd : mp.U;
        mp.Mf = gap ? mp.Nb : mp.Mb;
        mp.Vf = mp.V;
    }
    int64_t chol = std::max<int64_t>(mp.U, mp.V);
    for (const MpsSec *s : {&mp.A, &mp.B, &mp.G, &mp.O})
        if (s->comp) chol = std::max(chol, s->x * s->y);
    if (chol > MPS_CHOL_MAX)
        return fail(TNSLQ_E_ARG, "a factored matrix would be %lld wide (at most %lld)", (long long)chol,
                    (long long)MPS_CHOL_MAX);
    for (int k = 0; k < 4; ++k) {
        if (serr[k] == 1)
            return fail(TNSLQ_E_ARG, "%s: the explicit section would exceed 2^31 entries%s", sname[k],
                        secs[k]->comp ? " (the transfer route reaches it)" : "");
        if (serr[k] == 2) return fail(TNSLQ_E_ARG, "%s: the transfer sweep would exceed 2^32 entries", sname[k]);
    }
    mp.gmax = std::max<int64_t>(1, chol * chol);
    for (const MpsSec *s : {&mp.A, &mp.B, &mp.G, &mp.O}) {
        mp.smax = std::max(mp.smax, s->smax);
        mp.tmax = std::max(mp.tmax, s->tmax);
        mp.amax = std::max(mp.amax, s->amax);
    }
    mp.q[0] = (int)ceil_pow2_log(mp.kA);
    mp.q[1] = (int)ceil_pow2_log(mp.kB);
    mp.q[2] = (int)ceil_pow2_log(mp.Up * mp.Vf);
    if (!dense) {
        if (mp.kA * mp.kB > (int64_t(1) << 32))
            return fail(TNSLQ_E_ARG, "d_A' d_B' = %lld exceeds 2^32", (long long)(mp.kA * mp.kB));
        if (!net && (mp.kA * mp.Up > INT32_MAX || mp.kB * mp.Vf > INT32_MAX || mp.Up * mp.Mf > INT32_MAX ||
                     mp.Mf * mp.Vf > INT32_MAX || mp.kB * mp.Mf > INT32_MAX))
            return fail(TNSLQ_E_ARG, "the blocks' factors exceed 2^31 rows or columns");
    } else if (mp.q[0] + mp.q[1] + mp.q[2] > 32)
        return fail(TNSLQ_E_ARG, "the effective state would need %d qubits (at most 32)", mp.q[0] + mp.q[1] + mp.q[2]);
    size_t o = 0;
    auto take = [&](int64_t n) {
        size_t r = o;
        o += up((size_t)std::max<int64_t>(n, 1) * 16);
        return r;
    };
    const int64_t e2 = mp.closed ? 1 : mp.maxb * mp.maxb;
    mp.off_El[0] = take(e2);
    mp.off_El[1] = take(e2);
    mp.off_Er[0] = take(e2);
    mp.off_Er[1] = take(e2);
    mp.off_S[0] = take(mp.smax);
    mp.off_S[1] = take(mp.smax);
    mp.off_S[2] = take(mp.smax);
    mp.off_SA = take(mp.A.tr ? 1 : mp.U * mp.A.p * mp.Mb);
    mp.off_SB = take(mp.B.tr ? 1 : mp.Nb * mp.B.p * mp.V);
    mp.off_SG = take(gap && !mp.G.tr ? mp.Mb * mp.G.p * mp.Nb : 1);
    mp.off_SO = take(!mp.O.sites.empty() && !mp.O.tr ? mp.V * mp.O.p * mp.U : 1);
    mp.off_G = take(mp.gmax);
    mp.off_RA = take(mp.kA * mp.U * mp.Mb);
    mp.off_RB = take(mp.kB * mp.Nb * mp.V);
    const bool pq = dense || !net;   // the factors P, Q are built
    mp.off_RBp = take(mp.closed || !pq ? 1 : mp.kB * mp.Nb * mp.V);
    mp.off_W = take(gap ? mp.Mb * mp.Nb * mp.Wd : 1);
    mp.off_Z = take(mp.closed ? mp.V * mp.U * mp.Zd : 1);
    mp.off_T1 = take(gap && pq ? mp.kA * mp.U * mp.Nb * mp.Wd : 1);
    mp.off_T = take(dense ? mp.kA * mp.Up * mp.kB * mp.Vf : 1);
    mp.off_P = take((gap || mp.closed) && pq ? mp.kA * mp.Up * mp.Mf : 1);
    mp.off_Q2 = take(mp.closed && pq ? mp.kB * mp.Mf * mp.Vf : 1);
    mp.off_Q2p = take(mp.closed && pq ? mp.kB * mp.Mf * mp.Vf : 1);
    int64_t tenv = 0;   // the environment sweeps' scratch: one site tensor and one environment
    if (!mp.closed)
        for (int i = 0; i < L; ++i)
            if (i < mp.a0 || i >= mp.b1) tenv = std::max<int64_t>(tenv, (mp.off[i + 1] - mp.off[i]) + e2);
    mp.off_TT = take(tenv);
    const bool sweep = mp.A.tr || mp.B.tr || mp.G.tr || mp.O.tr;
    mp.off_Tt[0] = take(sweep ? mp.tmax : 1);
    mp.off_Tt[1] = take(sweep ? mp.tmax : 1);
    mp.off_At = take(sweep ? mp.amax : 1);
    mp.off_part = o;
    o += up(257 * 8);
    mp.off_fail = o;   // four flags, then at byte 64 the factorisations' scratch double, at 72 the sweeps'
    o += up(64 + 16);
    mp.total = o;
    return TNSLQ_OK;
}

// Contract the listed sites (consecutive along the ring) onto the running
// section S (rows r = left bond x physical so far, columns = bond), starting
// from S0 (rows0 x the first site's left bond); the result lands in `out`.
int mps_section(const MpsPlan &mp, const double2 *T, const double2 *S0, int64_t rows0, const int *sites, int ns,
                double2 *out, double2 *scratch0, double2 *scratch1, hipStream_t st) {
    const double2 *cur = S0;
    int64_t rows = rows0;
    for (int k = 0; k < ns; ++k) {
        const int i = sites[k];
        const int64_t z = mp.bond[i], py = (int64_t)mp.p[i] * mp.bond[i + 1];
        double2 *dst = k + 1 == ns ? out : (k % 2 ? scratch1 : scratch0);
        TNSLQ_HIP(launch_zgemm(0, 0, cur, T + mp.off[i], dst, (int)rows, (int)py, (int)z, z, py, py, 1, 0, 0, 0, st));
        cur = dst;
        rows *= mp.p[i];
    }
    return TNSLQ_OK;
}

// The explicit section S[x][phys][y] of s (x = its left bond): the first
// site's tensor itself when it is alone, else contracted into `out`.
int mps_section_of(const MpsPlan &mp, const double2 *T, const MpsSec &s, double2 *out, double2 *scratch0,
                   double2 *scratch1, hipStream_t st, const double2 **S) {
    const int i0 = s.sites.front();
    if (s.sites.size() == 1) {
        *S = T + mp.off[i0];
        return TNSLQ_OK;
    }
    *S = out;
    return mps_section(mp, T, T + mp.off[i0], s.x * mp.p[i0], s.sites.data() + 1, (int)s.sites.size() - 1, out,
                       scratch0, scratch1, st);
}

// The transfer matrix of the section s, T[(x, x')][y'][y], with X (x x x)
// absorbed on its left bond when not null; returns the buffer holding it.
double2 *mps_sweep(const MpsPlan &mp, const double2 *T, const MpsSec &s, const double2 *X, char *ws, hipStream_t st,
                   int &rc) {
    double2 *cur = (double2 *)(ws + mp.off_Tt[0]), *nxt = (double2 *)(ws + mp.off_Tt[1]);
    double2 *A = (double2 *)(ws + mp.off_At);
    double *tscr = (double *)(ws + mp.off_fail + 72);
    rc = TNSLQ_OK;
    hipError_t e = launch_transfer_start(X, s.x, cur, tscr, st);
    for (size_t k = 0; e == hipSuccess && k < s.sites.size(); ++k) {
        const int i = s.sites[k];
        e = launch_transfer_step(cur, T + mp.off[i], s.x, mp.bond[i], mp.p[i], mp.bond[i + 1], nxt, A, tscr, st);
        std::swap(cur, nxt);
    }
    if (e != hipSuccess) rc = fail(TNSLQ_E_DEVICE, "transfer sweep: %s", hipGetErrorString(e));
    return cur;
}

// R[k][(l, r)] for a section S[l][phys][r]: S itself with its first two axes
// exchanged, or (compressed) R = L^dagger with L L^dagger = S^dagger S over
// the physical index.  The Gram product's reduction over the physical index
// is split until it fills the chip (partials in `part`, part_cap entries),
// then summed.
int mps_vertical(const double2 *S, int64_t l, int64_t ph, int64_t r, int comp, double2 *R, double2 *tmp, double2 *G,
                 double2 *part, int64_t part_cap, int *failp, double *dscr, hipStream_t st) {
    if (!comp) {
        TNSLQ_HIP(launch_swap01(S, 1, l, ph, r, 0, R, st));
        return TNSLQ_OK;
    }
    const int64_t n = l * r;
    TNSLQ_HIP(launch_swap01(S, 1, l, ph, r, 0, tmp, st));   // [phys][(l r)]
    const int64_t tiles = ((n + 63) / 64) * ((n + 63) / 64);
    int ks = 1;
    while (tiles * ks < 1024 && ph / (2 * ks) >= 256 && 2 * ks * n * n <= part_cap && 2 * ks <= 64) ks *= 2;
    if (ks > 1) {
        TNSLQ_HIP(launch_zgemm(2, 0, tmp, tmp, part, (int)n, (int)n, (int)ph, n, n, n, 1, 0, 0, 0, st, 0, ks, n * n));
        TNSLQ_HIP(launch_sum_splits(part, ks, n * n, G, st));
    } else {
        TNSLQ_HIP(launch_zgemm(2, 0, tmp, tmp, G, (int)n, (int)n, (int)ph, n, n, n, 1, 0, 0, 0, st));
    }
    TNSLQ_HIP(launch_cholesky(G, (int)n, failp, dscr, st));
    TNSLQ_HIP(launch_swap01(G, 1, n, n, 1, 1, R, st));
    return TNSLQ_OK;
}

// R[k][(x, y)] = L^dagger for the Gram matrix of a section given by its
// transfer matrix Tr[x][x'][y'][y]: G[x][y][x'][y'] = Tr[x'][x][y][y'].
int mps_vertical_transfer(const double2 *Tr, int64_t x, int64_t y, double2 *R, double2 *G, int *failp, double *dscr,
                          hipStream_t st) {
    const int64_t d[4] = {x, x, y, y};
    const int perm[4] = {1, 2, 0, 3};
    TNSLQ_HIP(launch_permute4(Tr, d, perm, G, st));
    TNSLQ_HIP(launch_cholesky(G, (int)(x * y), failp, dscr, st));
    TNSLQ_HIP(launch_swap01(G, 1, x * y, x * y, 1, 1, R, st));
    return TNSLQ_OK;
}

// F[(x, y)][f] with F F^dagger = the section's matrix sum_s S[x][s][y]
// conj(S[x'][s][y']) = Tr[x][x'][y'][y] (a traced gap or outer section), in
// place in F (x y x y entries).
int mps_trace_factor_transfer(const double2 *Tr, int64_t x, int64_t y, double2 *F, int *failp, double *dscr,
                              hipStream_t st) {
    const int64_t d[4] = {x, x, y, y};
    const int perm[4] = {0, 3, 1, 2};
    TNSLQ_HIP(launch_permute4(Tr, d, perm, F, st));
    TNSLQ_HIP(launch_cholesky(F, (int)(x * y), failp, dscr, st));
    return TNSLQ_OK;
}

// F[x][y][f] for an explicit traced section S[x][g][y]: S with its last two
// axes exchanged when g <= x y (F holds x y g entries), else the Cholesky
// factor of sum_g S[x][g][y] conj(S[x'][g][y']) (F holds (x y)^2 entries; the
// exchanged section goes to tmp, x g y entries, the Gram matrix to G).
int mps_trace_factor(const double2 *S, int64_t x, int64_t g, int64_t y, bool comp, double2 *F, double2 *tmp,
                     double2 *G, int *failp, double *dscr, hipStream_t st) {
    if (!comp) {
        TNSLQ_HIP(launch_swap01(S, x, g, y, 1, 0, F, st));   // [x][y][g]
        return TNSLQ_OK;
    }
    const int64_t n = x * y;
    TNSLQ_HIP(launch_swap01(S, x, g, y, 1, 0, tmp, st));
    TNSLQ_HIP(launch_zgemm(0, 2, tmp, tmp, G, (int)n, (int)n, (int)g, g, g, n, 1, 0, 0, 0, st));
    TNSLQ_HIP(launch_cholesky(G, (int)n, failp, dscr, st));
    TNSLQ_HIP(hipMemcpyAsync(F, G, (size_t)n * n * 16, hipMemcpyDeviceToDevice, st));
    return TNSLQ_OK;
}

// The factors of the effective state psi[a][b][(u', v')] = sum_m P[a][u'][m]
// Q[b][m][v']:
//   open, adjacent:  P = R_A, u' = u, m the bond between the blocks, v' = v;
//   open, gap:       P[a][(u, w)][n] = sum_m R_A[a][u][m] W[m][n][w];
//   ring:            P[a][w][(n, u)] = sum_m R_A[a][u][m] W[m][n][w] (W the
//                    identity when adjacent), Q[b][(n, u)][z] = sum_v
//                    R_B[b][n][v] Z[v][u][z], v' = z.
// Qp is Q with its first two axes exchanged, [m][b][v'].  The network form
// keeps the pieces: R_A[a][u][m], R_B[b][n][v], W[(m, n)][w] (a gap),
// Z[(v, u)][z] (a ring).
struct MpsFactors {
    double2 *P;
    const double2 *Q, *Qp;
    int64_t kA, Up, M, kB, V;
    double2 *RA;
    const double2 *RB, *W, *Z;
    int64_t U, Mb, Nb, Vb, Wd, Zd;
};

// net: stop once the pieces of the network form are built (no P, Q).
int mps_build(const MpsPlan &mp, const double2 *T, char *ws, hipStream_t st, MpsFactors &f, bool net = false) {
    int rc;
    auto buf = [&](size_t off) { return (double2 *)(ws + off); };
    int *failp = (int *)(ws + mp.off_fail);
    double *dscr = (double *)(ws + mp.off_fail + 64);   // the factorisations' largest diagonal entry
    TNSLQ_HIP(launch_zero(failp, 16, st));
    static const double2 one = {1.0, 0.0};
    double2 *s0 = buf(mp.off_S[0]), *s1 = buf(mp.off_S[1]), *s2 = buf(mp.off_S[2]);
    const double2 *X = nullptr, *Y = nullptr;
    double2 *Xt = nullptr;
    if (!mp.closed) {
        // traced environments: E_L on the bond entering A, E_R on the bond leaving B
        double2 *El = buf(mp.off_El[0]), *Eln = buf(mp.off_El[1]);
        TNSLQ_HIP(hipMemcpyAsync(El, &one, sizeof one, hipMemcpyHostToDevice, st));
        for (int i = 0; i < mp.a0; ++i) {
            TNSLQ_HIP(
                launch_transfer(1, El, T + mp.off[i], mp.bond[i], mp.p[i], mp.bond[i + 1], Eln, buf(mp.off_TT), st));
            std::swap(El, Eln);
        }
        double2 *Er = buf(mp.off_Er[0]), *Ern = buf(mp.off_Er[1]);
        TNSLQ_HIP(hipMemcpyAsync(Er, &one, sizeof one, hipMemcpyHostToDevice, st));
        for (int i = mp.L - 1; i >= mp.b1; --i) {
            TNSLQ_HIP(
                launch_transfer(0, Er, T + mp.off[i], mp.bond[i], mp.p[i], mp.bond[i + 1], Ern, buf(mp.off_TT), st));
            std::swap(Er, Ern);
        }
        TNSLQ_HIP(launch_cholesky(El, (int)mp.U, failp, dscr, st));       // X[x][u]
        TNSLQ_HIP(launch_cholesky(Er, (int)mp.V, failp + 1, dscr, st));   // Y[y][v]
        X = El;
        Y = Er;
        Xt = Eln;
        TNSLQ_HIP(launch_swap01(El, 1, mp.U, mp.U, 1, 0, Xt, st));        // X^T (rows u, columns x)
    }
    // block A: R_A[kA][u][m]
    if (mp.A.tr) {
        double2 *Ta = mps_sweep(mp, T, mp.A, X, ws, st, rc);
        if (rc) return rc;
        if ((rc = mps_vertical_transfer(Ta, mp.U, mp.Mb, buf(mp.off_RA), buf(mp.off_G), failp + 2, dscr, st)))
            return rc;
    } else {
        const double2 *SA;
        if (X) {
            if ((rc = mps_section(mp, T, Xt, mp.U, mp.A.sites.data(), (int)mp.A.sites.size(), buf(mp.off_SA), s0, s1,
                                  st)))
                return rc;
            SA = buf(mp.off_SA);
        } else if ((rc = mps_section_of(mp, T, mp.A, buf(mp.off_SA), s0, s1, st, &SA))) {
            return rc;
        }
        if ((rc = mps_vertical(SA, mp.U, mp.A.p, mp.Mb, mp.A.comp, buf(mp.off_RA), s0, buf(mp.off_G), s1, mp.smax,
                               failp + 2, dscr, st)))
            return rc;
    }
    // block B: R_B[kB][n][v]
    if (mp.B.tr) {
        double2 *Tb = mps_sweep(mp, T, mp.B, nullptr, ws, st, rc);
        if (rc) return rc;
        if (Y) {
            double2 *Tn = Tb == buf(mp.off_Tt[0]) ? buf(mp.off_Tt[1]) : buf(mp.off_Tt[0]);
            TNSLQ_HIP(launch_transfer_absorb_right(Tb, Y, mp.Nb, mp.V, mp.V, Tn, buf(mp.off_At),
                                                   (double *)(ws + mp.off_fail + 72), st));
            Tb = Tn;
        }
        if ((rc = mps_vertical_transfer(Tb, mp.Nb, mp.V, buf(mp.off_RB), buf(mp.off_G), failp + 3, dscr, st)))
            return rc;
    } else {
        const double2 *SB;
        if ((rc = mps_section_of(mp, T, mp.B, s2, s0, s1, st, &SB))) return rc;
        if (Y) {
            TNSLQ_HIP(launch_zgemm(0, 0, SB, Y, buf(mp.off_SB), (int)(mp.Nb * mp.B.p), (int)mp.V, (int)mp.V, mp.V,
                                   mp.V, mp.V, 1, 0, 0, 0, st));
            SB = buf(mp.off_SB);
        }
        if ((rc = mps_vertical(SB, mp.Nb, mp.B.p, mp.V, mp.B.comp, buf(mp.off_RB), s0, buf(mp.off_G), s1, mp.smax,
                               failp + 3, dscr, st)))
            return rc;
    }
    const bool gap = mp.b0 > mp.a1;
    // the gap: W[m][n][w]
    if (gap) {
        if (mp.G.tr) {
            double2 *Tg = mps_sweep(mp, T, mp.G, nullptr, ws, st, rc);
            if (rc) return rc;
            if ((rc = mps_trace_factor_transfer(Tg, mp.Mb, mp.Nb, buf(mp.off_W), failp + 3, dscr, st))) return rc;
        } else {
            const double2 *SG;
            if ((rc = mps_section_of(mp, T, mp.G, buf(mp.off_SG), s0, s1, st, &SG))) return rc;
            if ((rc = mps_trace_factor(SG, mp.Mb, mp.G.p, mp.Nb, mp.G.comp, buf(mp.off_W), s2, buf(mp.off_G),
                                       failp + 3, dscr, st)))
                return rc;
        }
    }
    // a ring's outer section: Z[v][u][z]
    if (mp.closed) {
        if (mp.O.sites.empty()) {
            TNSLQ_HIP(launch_identity(buf(mp.off_Z), mp.V, st));
        } else if (mp.O.tr) {
            double2 *To = mps_sweep(mp, T, mp.O, nullptr, ws, st, rc);
            if (rc) return rc;
            if ((rc = mps_trace_factor_transfer(To, mp.V, mp.U, buf(mp.off_Z), failp + 3, dscr, st))) return rc;
        } else {
            const double2 *SO;
            if ((rc = mps_section_of(mp, T, mp.O, buf(mp.off_SO), s0, s1, st, &SO))) return rc;
            if ((rc = mps_trace_factor(SO, mp.V, mp.O.p, mp.U, mp.O.comp, buf(mp.off_Z), s2, buf(mp.off_G),
                                       failp + 3, dscr, st)))
                return rc;
        }
    }
    f.kA = mp.kA;
    f.kB = mp.kB;
    f.Up = mp.Up;
    f.M = mp.Mf;
    f.V = mp.Vf;
    f.RA = buf(mp.off_RA);
    f.RB = buf(mp.off_RB);
    f.W = gap ? buf(mp.off_W) : nullptr;
    f.Z = mp.closed ? buf(mp.off_Z) : nullptr;
    f.U = mp.U;
    f.Mb = mp.Mb;
    f.Nb = mp.Nb;
    f.Vb = mp.V;
    f.Wd = mp.Wd;
    f.Zd = mp.Zd;
    if (net) {
        f.P = nullptr;
        f.Q = f.Qp = nullptr;
        return TNSLQ_OK;
    }
    // T1[(kA, u)][(n, w)] = sum_m R_A[(kA, u)][m] W[m][(n, w)]
    const int64_t nrow = mp.kA * mp.U;
    if (gap)
        TNSLQ_HIP(launch_zgemm(0, 0, buf(mp.off_RA), buf(mp.off_W), buf(mp.off_T1), (int)nrow, (int)(mp.Nb * mp.Wd),
                               (int)mp.Mb, mp.Mb, mp.Nb * mp.Wd, mp.Nb * mp.Wd, 1, 0, 0, 0, st));
    if (!mp.closed) {
        TNSLQ_HIP(launch_swap01(buf(mp.off_RB), 1, mp.kB, mp.Nb, mp.V, 0, buf(mp.off_RBp), st));   // [n][kB][v]
        f.Q = buf(mp.off_RB);
        f.Qp = buf(mp.off_RBp);
        if (!gap) {
            f.P = buf(mp.off_RA);
        } else {
            TNSLQ_HIP(launch_swap01(buf(mp.off_T1), nrow, mp.Nb, mp.Wd, 1, 0, buf(mp.off_P), st));   // [(kA, u)][w][n]
            f.P = buf(mp.off_P);
        }
        return TNSLQ_OK;
    }
    // ring: Q[(kB, n)][(u, z)] = sum_v R_B[(kB, n)][v] Z[v][(u, z)], Qp = [(n, u)][kB][z]
    const int64_t uz = mp.U * mp.Zd;
    TNSLQ_HIP(launch_zgemm(0, 0, buf(mp.off_RB), buf(mp.off_Z), buf(mp.off_Q2), (int)(mp.kB * mp.Nb), (int)uz,
                           (int)mp.V, mp.V, uz, uz, 1, 0, 0, 0, st));
    TNSLQ_HIP(launch_swap01(buf(mp.off_Q2), 1, mp.kB, mp.Mf, mp.Zd, 0, buf(mp.off_Q2p), st));
    if (gap) {
        // P[a][w][n][u] = T1[a][u][n][w]
        const int64_t d[4] = {mp.kA, mp.U, mp.Nb, mp.Wd};
        const int perm[4] = {0, 3, 2, 1};
        TNSLQ_HIP(launch_permute4(buf(mp.off_T1), d, perm, buf(mp.off_P), st));
    } else {
        // P[a][m][u] = R_A[a][u][m] (w of size 1)
        TNSLQ_HIP(launch_swap01(buf(mp.off_RA), mp.kA, mp.U, mp.Mb, 1, 0, buf(mp.off_P), st));
    }
    f.P = buf(mp.off_P);
    f.Q = buf(mp.off_Q2);
    f.Qp = buf(mp.off_Q2p);
    return TNSLQ_OK;
}

// Read the factorisations' outcome (synchronises).
int mps_check(const MpsPlan &mp, char *ws, hipStream_t st) {
    int hf[4] = {0, 0, 0, 0};
    TNSLQ_HIP(hipMemcpyAsync(hf, ws + mp.off_fail, sizeof hf, hipMemcpyDeviceToHost, st));
    TNSLQ_HIP(hipStreamSynchronize(st));
    static const char *what[4] = {"left environment", "right environment", "block A", "block B or the gap"};
    for (int i = 0; i < 4; ++i)
        if (hf[i]) return fail(TNSLQ_E_NONFINITE, "%s: matrix to factor is not finite", what[i]);
    return TNSLQ_OK;
}

struct Ctx {
    Plan pl;
    char *ws;
    hipStream_t st;
    LzDims z;
    void *Paeb, *Pbea, *Xt, *Ups, *Ypart, *U1part;
    void *P1s, *P2s;
    void *Pabe, *Pabc, *Cd, *rho;
    double2 *Up, *U2, *Xs, *Xq, *Ym;
    const MpsPlan *mp = nullptr;     // factorised MPS operator: its factor construction
    MpsFactors mf{};
    double2 *Z1, *Z2, *Z2p, *Z3;     // complex64 in FP32
    float2 *P32, *Q32, *X32;
    double2 *Q, *w;
    double *alpha, *beta, *F, *G, *stats, *dotpart, *nrmpart, *hpart;
    double2 *h;
    int *steps;
    double *finf, *fsig, *fitout;
    float *feat;
    void *mlpws;
    std::vector<hipEvent_t> ev;
    int n_launch = 0;
    ~Ctx() {
        for (auto e : ev) (void)hipEventDestroy(e);
    }
    hipEvent_t event() {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        ev.push_back(e);
        return e;
    }
};

void bind(Ctx &c, void *ws, hipStream_t st) {
    Plan &pl = c.pl;
    c.ws = (char *)ws;
    c.st = st;
    c.Paeb = c.ws + pl.off_Paeb;
    c.Pbea = c.ws + pl.off_Pbea;
    c.Xt = c.ws + pl.off_Xt;
    c.Ups = c.ws + pl.off_Ups;
    c.Ypart = c.ws + pl.off_Ypart;
    c.U1part = pl.S1 > 1 ? c.ws + pl.off_U1part : nullptr;
    c.P1s = c.ws + pl.off_P1s;
    c.P2s = c.ws + pl.off_P2s;
    c.Up = (double2 *)(c.ws + pl.off_Up);
    c.U2 = (double2 *)(c.ws + pl.off_U2);
    c.Xs = (double2 *)(c.ws + pl.off_Xs);
    c.Xq = (double2 *)(c.ws + pl.off_Xq);
    c.Ym = (double2 *)(c.ws + pl.off_Ym);
    if (pl.stream) c.Paeb = c.Pbea = c.Xt = c.Ups = nullptr;
    c.Pabe = pl.expl ? c.ws + pl.off_Pabe : nullptr;
    c.Pabc = pl.expl ? c.ws + pl.off_Pabc : nullptr;
    c.Cd = pl.expl ? c.ws + pl.off_Cd : nullptr;
    c.rho = pl.expl ? c.ws + pl.off_rho : nullptr;
    if (pl.expl) c.Paeb = c.Pbea = c.Ups = nullptr;
    c.Z1 = (double2 *)(c.ws + pl.off_Z1);
    c.Z2 = (double2 *)(c.ws + pl.off_Z2);
    c.Z2p = (double2 *)(c.ws + pl.off_Z2p);
    c.Z3 = (double2 *)(c.ws + pl.off_Z3);
    c.P32 = (float2 *)(c.ws + pl.off_P32);
    c.Q32 = (float2 *)(c.ws + pl.off_Q32);
    c.X32 = (float2 *)(c.ws + pl.off_X32);
    if (pl.mpsf) c.Paeb = c.Pbea = c.Xt = c.Ups = nullptr;
    c.Q = (double2 *)(c.ws + pl.off_Q);
    c.w = (double2 *)(c.ws + pl.off_w);
    c.alpha = (double *)(c.ws + pl.off_alpha);
    c.beta = (double *)(c.ws + pl.off_beta);
    c.F = (double *)(c.ws + pl.off_F);
    c.G = (double *)(c.ws + pl.off_G);
    c.stats = (double *)(c.ws + pl.off_stats);
    c.dotpart = (double *)(c.ws + pl.off_red);
    c.nrmpart = c.dotpart + (size_t)pl.K * pl.nblk;
    c.hpart = (double *)(c.ws + pl.off_h);
    c.h = (double2 *)(c.ws + pl.off_h + (size_t)pl.K * (pl.m + 1) * pl.nblk * 16);
    c.steps = (int *)(c.ws + pl.off_steps);
    c.finf = (double *)(c.ws + pl.off_fit);
    c.fsig = c.finf + pl.K;
    c.fitout = c.fsig + pl.K;
    c.feat = (float *)(c.ws + pl.off_feat);
    c.mlpws = c.ws + pl.off_mlp;
    // the explicit form contracts the vectors over the whole index (a, b): its
    // transposed copy Xt has rows k and reduction index a d_B + b
    c.z = pl.expl ? LzDims{pl.dAB, 1, pl.dAB, pl.K, pl.m, pl.nblk} : LzDims{pl.dA, pl.dB, pl.dAB, pl.K, pl.m, pl.nblk};
}

// Regroup psi into both contraction layouts, and zero the padding of Xt and
// Ups along their reduction index (written nowhere else; padded rows need no
// clearing, their products land outside C).
// rho_AB = P P^dagger (Sec. V: the partial trace over E) as a dense n x n
// product in the accumulator type, from P[(a, b)][c] = psi regrouped as
// (A, B, E) and its conjugate, both as brick operands of precision `prec`.
int form_rho(const Plan &pl, int prec, const void *psi, void *Pabe, void *Pabc, void *Cd, hipStream_t st) {
    const int64_t n = pl.dAB, dE = pl.dE;
    if (pl.mixed) {
        TNSLQ_HIP(launch_permute_mixed(prec, pl.dtype, psi, Pabe, pl.md, 0, st));
        TNSLQ_HIP(launch_permute_mixed(prec, pl.dtype, psi, Pabc, pl.md, 1, st));
    } else {
        const PermDesc abe = perm_for(pl, pl.qa, pl.nA, pl.qb, pl.nB, pl.qe, pl.nE);
        TNSLQ_HIP(launch_permute(prec, pl.dtype, psi, Pabe, n, dE, abe, 0, st));
        TNSLQ_HIP(launch_permute(prec, pl.dtype, psi, Pabc, n, dE, abe, 1, st));
    }
    GemmDesc g{};
    g.A = Pabe;
    g.B = Pabc;
    g.C = Cd;
    g.M = n;
    g.N = n;
    g.Kr = dE;
    g.nst = brick_stages(prec, dE);
    g.S = 1;
    g.out_mode = 1;   // C[i][j] at i n + j
    g.cnb_log2 = 0;
    g.cni_log2 = 0;
    g.ldc = n;
    g.cbs = 1;
    g.c_split = 0;
    TNSLQ_HIP(launch_gemm(prec, g, st));
    return TNSLQ_OK;
}

// The network form (psi is the chain's tensors): R_A, R_B and the traced
// sections' matrices E_W = W W^dagger, E_Z = Z Z^dagger regrouped for the
// matvec, then R_A scaled so that the effective state has norm 1:
//   ||psi||^2 = sum GA[u'][m'][u][m] E_W[m][n][m'][n'] HB[n'][v'][n][v]
//               E_Z[v][u][v'][u']
// with GA = R_A^dagger R_A, HB = R_B^dagger R_B (open chains: E_Z the
// identity on (u, v); adjacent blocks: E_W the identity, n = m).
int net_layout(Ctx &c, const void *psi) {
    const Plan &pl = c.pl;
    int rc;
    char *mws = c.ws + pl.off_mps;
    if ((rc = mps_build(*c.mp, (const double2 *)psi, mws, c.st, c.mf, true))) return rc;
    const MpsFactors &f = c.mf;
    if (f.kA != pl.dA || f.kB != pl.dB || f.U != pl.nU || f.Mb != pl.nM || f.Nb != pl.nN || f.Vb != pl.nV)
        return fail(TNSLQ_E_ARG, "network shapes differ from the plan");
    const int64_t U = pl.nU, M = pl.nM, N = pl.nN, V = pl.nV, UM = U * M, NV = N * V, MN = M * N, UV = U * V;
    const NetBufs nb = net_bufs(pl);
    char *base = c.ws + pl.off_net;
    auto at = [&](size_t off) { return (double2 *)(base + off); };
    double2 *x0 = at(nb.x[0]), *x1 = at(nb.x[1]), *x2 = at(nb.x[2]), *x3 = at(nb.x[3]);
    double *nrm = (double *)(c.ws + pl.off_nrm);
    const int kA = (int)f.kA, kB = (int)f.kB;
    if (pl.ngap) {
        // E_W[(m, n)][(m', n')] in x2, regrouped as [m][n'][m'][n]
        TNSLQ_HIP(launch_zgemm(0, 2, f.W, f.W, x2, (int)MN, (int)MN, (int)f.Wd, f.Wd, f.Wd, MN, 1, 0, 0, 0, c.st));
        const int64_t d[4] = {M, N, M, N};
        const int perm[4] = {0, 3, 2, 1};
        TNSLQ_HIP(launch_permute4(x2, d, perm, at(nb.ewp), c.st));
    }
    if (pl.nring) {
        // E_Z[(v, u)][(v', u')] in x3, regrouped as [u][v'][v][u']
        TNSLQ_HIP(launch_zgemm(0, 2, f.Z, f.Z, x3, (int)UV, (int)UV, (int)f.Zd, f.Zd, f.Zd, UV, 1, 0, 0, 0, c.st));
        const int64_t d[4] = {V, U, V, U};
        const int perm[4] = {1, 2, 0, 3};
        TNSLQ_HIP(launch_permute4(x3, d, perm, at(nb.ezp), c.st));
    }
    // GA[(u', m')][(u, m)] in x0, as [(u', u)][(m, m')] in x1
    TNSLQ_HIP(launch_zgemm(2, 0, f.RA, f.RA, x0, (int)UM, (int)UM, kA, UM, UM, UM, 1, 0, 0, 0, c.st));
    {
        const int64_t d[4] = {U, M, U, M};
        const int perm[4] = {0, 2, 3, 1};
        TNSLQ_HIP(launch_permute4(x0, d, perm, x1, c.st));
    }
    // F1[(u', u)][(n, n')] = sum_{m, m'} GA E_W
    double2 *F1 = x1, *fr0 = x0, *fr1 = x2;
    if (pl.ngap) {
        const int64_t d[4] = {M, N, M, N};
        const int perm[4] = {0, 2, 1, 3};   // E_W as [(m, m')][(n, n')]
        TNSLQ_HIP(launch_permute4(x2, d, perm, x0, c.st));
        TNSLQ_HIP(launch_zgemm(0, 0, x1, x0, x2, (int)(U * U), (int)(N * N), (int)(M * M), M * M, N * N, N * N, 1, 0,
                               0, 0, c.st));
        F1 = x2;
        fr0 = x0;
        fr1 = x1;
    }
    // HB[(n', v')][(n, v)], as [(n, n')][(v', v)]; F2[(u', u)][(v', v)] = F1 HB
    TNSLQ_HIP(launch_zgemm(2, 0, f.RB, f.RB, fr0, (int)NV, (int)NV, kB, NV, NV, NV, 1, 0, 0, 0, c.st));
    {
        const int64_t d[4] = {N, V, N, V};
        const int perm[4] = {2, 0, 1, 3};
        TNSLQ_HIP(launch_permute4(fr0, d, perm, fr1, c.st));
    }
    double2 *F2 = fr0;
    TNSLQ_HIP(launch_zgemm(0, 0, F1, fr1, F2, (int)(U * U), (int)(V * V), (int)(N * N), N * N, V * V, V * V, 1, 0, 0,
                           0, c.st));
    if (pl.nring) {
        // ||psi||^2 = Re sum F2[u'][u][v'][v] conj E_Z[v'][u'][v][u]
        const int64_t d[4] = {V, U, V, U};
        const int perm[4] = {1, 3, 0, 2};
        TNSLQ_HIP(launch_permute4(x3, d, perm, fr1, c.st));
        TNSLQ_HIP(launch_normalise_factor(F2, fr1, UV * UV, nrm, f.RA, f.kA * UM, c.st));
    } else {
        // ||psi||^2 = sum_{u, v} F2[u][u][v][v]
        TNSLQ_HIP(launch_trace_pairs(F2, U, V, nrm, c.st));
        TNSLQ_HIP(launch_scale_rsqrt(f.RA, f.kA * UM, nrm, c.st));
    }
    if (pl.prec == TNSLQ_FP32) {
        TNSLQ_HIP(launch_to_c64(f.RA, f.kA * UM, c.P32, c.st));
        TNSLQ_HIP(launch_to_c64(f.RB, f.kB * NV, c.Q32, c.st));
        if (pl.ngap) TNSLQ_HIP(launch_to_c64(at(nb.ewp), MN * MN, (float2 *)(base + nb.ew32), c.st));
        if (pl.nring) TNSLQ_HIP(launch_to_c64(at(nb.ezp), UV * UV, (float2 *)(base + nb.ez32), c.st));
    }
    return mps_check(*c.mp, mws, c.st);
}

int do_layout(Ctx &c, const void *psi) {
    const Plan &pl = c.pl;
    if (pl.mpsf && pl.mnet) return net_layout(c, psi);
    if (pl.mpsf) {
        // the factors P and Q of the two blocks (psi is the chain's tensors),
        // then psi = P Q normalised through P: ||psi||^2 = Re sum Ahat conj(C)
        // with Ahat = P^dagger P and C = Qp Qp^dagger over the bond index m
        int rc;
        char *mws = c.ws + pl.off_mps;
        if ((rc = mps_build(*c.mp, (const double2 *)psi, mws, c.st, c.mf))) return rc;
        MpsFactors &f = c.mf;
        if (f.kA != pl.dA || f.kB != pl.dB || f.Up != pl.mUp || f.M != pl.mM || f.V != pl.mV)
            return fail(TNSLQ_E_ARG, "factor shapes differ from the plan");
        double2 *Ah = (double2 *)(c.ws + pl.off_nrm), *Cq = Ah + pl.mM * pl.mM;
        double *nrm = (double *)(Cq + pl.mM * pl.mM);
        const int M = (int)f.M;
        const int64_t rowsP = f.kA * f.Up, colsQ = f.kB * f.V, mm = (int64_t)M * M;
        // M x M outputs over long reductions (k^2 chi terms): split until the
        // products fill the chip, partials in the still unused intermediate Z2
        const int64_t tiles = ((M + 63) / 64) * ((M + 63) / 64);
        const int64_t cap = (int64_t)(pl.kc * pl.mUp * pl.mM * pl.mM * pl.mV * (pl.prec == TNSLQ_FP32 ? 8 : 16) / 16);
        auto splits = [&](int64_t K) {
            int ks = 1;
            while (tiles * ks < 1024 && K / (2 * ks) >= 256 && 2 * ks * mm <= cap && 2 * ks <= 1024) ks *= 2;
            return ks;
        };
        const int ksA = splits(rowsP), ksC = splits(colsQ);
        if (ksA > 1) {
            TNSLQ_HIP(launch_zgemm(2, 0, f.P, f.P, c.Z2, M, M, (int)rowsP, M, M, M, 1, 0, 0, 0, c.st, 0, ksA, mm));
            TNSLQ_HIP(launch_sum_splits(c.Z2, ksA, mm, Ah, c.st));
        } else {
            TNSLQ_HIP(launch_zgemm(2, 0, f.P, f.P, Ah, M, M, (int)rowsP, M, M, M, 1, 0, 0, 0, c.st));
        }
        if (ksC > 1) {
            TNSLQ_HIP(
                launch_zgemm(0, 2, f.Qp, f.Qp, c.Z2, M, M, (int)colsQ, colsQ, colsQ, M, 1, 0, 0, 0, c.st, 0, ksC, mm));
            TNSLQ_HIP(launch_sum_splits(c.Z2, ksC, mm, Cq, c.st));
        } else {
            TNSLQ_HIP(launch_zgemm(0, 2, f.Qp, f.Qp, Cq, M, M, (int)colsQ, colsQ, colsQ, M, 1, 0, 0, 0, c.st));
        }
        TNSLQ_HIP(launch_normalise_factor(Ah, Cq, (int64_t)M * M, nrm, f.P, rowsP * M, c.st));
        if (pl.prec == TNSLQ_FP32) {
            TNSLQ_HIP(launch_to_c64(f.P, rowsP * M, c.P32, c.st));
            TNSLQ_HIP(launch_to_c64(f.Q, f.kB * M * f.V, c.Q32, c.st));
        }
        return mps_check(*c.mp, mws, c.st);
    }
    if (pl.expl) {
        // intermediary (iii): rho^{T_B} formed once, as the brick operand of
        // every later matvec
        int rc;
        if ((rc = form_rho(pl, pl.prec, psi, c.Pabe, c.Pabc, c.Cd, c.st))) return rc;
        TNSLQ_HIP(launch_pt_bricks(pl.prec, pl.prec == TNSLQ_FP64, c.Cd, pl.dAB, pl.dB, c.rho, pl.nst_rho, c.st));
        if (pl.dAB % brick_epr(pl.prec))
            TNSLQ_HIP(launch_zero(c.Xt, brick_bytes(pl.prec, pl.K, pl.dAB), c.st));
        return TNSLQ_OK;
    }
    if (pl.stream && pl.fused) {
        // (E, A, B), B fastest: environment slab c is a contiguous d_A x d_B
        // matrix (the panel layout with 512 columns is row-major)
        const PermDesc eab = perm_for(pl, pl.qe, pl.nE, pl.qa, pl.nA, pl.qb, pl.nB);
        TNSLQ_HIP(launch_regroup(pl.dtype, psi, c.P1s, pl.D / 512, 512, eab, c.st));
        return TNSLQ_OK;
    }
    if (pl.stream) {
        // (A; E, B): rows a', columns (c, b); (E, B; A): rows (c, b'), columns a
        int eb[TNSLQ_MAX_QUBITS];
        for (int i = 0; i < pl.nE; ++i) eb[i] = pl.qe[i];
        for (int i = 0; i < pl.nB; ++i) eb[pl.nE + i] = pl.qb[i];
        const PermDesc p1 = perm_two(pl.L, pl.qa, pl.nA, eb, pl.nE + pl.nB);
        const PermDesc p2 = perm_two(pl.L, eb, pl.nE + pl.nB, pl.qa, pl.nA);
        TNSLQ_HIP(launch_regroup(pl.dtype, psi, c.P1s, pl.dA, pl.dE * pl.dB, p1, c.st));
        TNSLQ_HIP(launch_regroup(pl.dtype, psi, c.P2s, pl.dE * pl.dB, pl.dA, p2, c.st));
        return TNSLQ_OK;
    }
    PermDesc aeb = perm_for(pl, pl.qa, pl.nA, pl.qe, pl.nE, pl.qb, pl.nB);
    PermDesc bea = perm_for(pl, pl.qb, pl.nB, pl.qe, pl.nE, pl.qa, pl.nA);
    TNSLQ_HIP(launch_permute(pl.prec, pl.dtype, psi, c.Paeb, pl.dA, pl.dE * pl.dB, aeb, 0, c.st));
    TNSLQ_HIP(launch_permute(pl.prec, pl.dtype, psi, c.Pbea, pl.dB * pl.dE, pl.dA, bea, 1, c.st));
    const int64_t epr = brick_epr(pl.prec);
    if (pl.dA % epr)
        TNSLQ_HIP(launch_zero(c.Xt, brick_bytes(pl.prec, (int64_t)pl.K * pl.dB, pl.dA), c.st));
    if ((pl.dE * pl.dB) % epr)
        TNSLQ_HIP(launch_zero(c.Ups, brick_bytes(pl.prec, (int64_t)pl.kc * pl.dB, pl.dE * pl.dB), c.st));
    return TNSLQ_OK;
}

// The streaming form of both contractions for all K probes (Sec. V Eq. 4,
// intermediary (i)), from FP64 vectors xq[k][a dB + b]:
//   Xq[(k, b')][a']        = xq[k][a' dB + b']
//   Up[s][(k, b')][(c, b)] = sum_{a' in split s} conj psi[a', c, b] Xq[(k, b')][a']
//   U2[(k, b)][(c, b')]    = sum_s Up[s][(k, b')][(c, b)]
//   Yt[s][(k, b)][a]       = sum_{(c, b') in split s} psi[a, c, b'] U2[(k, b)][(c, b')]
//   Ym[k][a dB + b]        = sum_s Yt[s][(k, b)][a]
// Both passes read their vectors and write their outputs contiguously, the
// column MAC's plain form.
int stream_contract(Ctx &c, const double2 *xq, hipEvent_t e1, hipEvent_t e2) {
    const Plan &pl = c.pl;
    if (pl.fused) {
        // both contractions in one read of psi; the Lanczos pass (or the
        // matvec's reduction) sums the blocks' partials
        if (e1) TNSLQ_HIP(hipEventRecord(e1, c.st));
        TNSLQ_HIP(launch_pt_fused(c.P1s, xq, pl.dA, pl.dB, pl.K, pl.dE, FUSED_BLOCKS, (double2 *)c.Ypart, c.st));
        if (e2) TNSLQ_HIP(hipEventRecord(e2, c.st));
        c.n_launch++;
        return TNSLQ_OK;
    }
    const int64_t ncol = pl.dE * pl.dB;
    const int nv = pl.K * (int)pl.dB;
    TNSLQ_HIP(launch_vectors_by_b(xq, pl.K, pl.dA, pl.nB, c.Xq, c.st));
    TNSLQ_HIP(launch_colmac(pl.dtype, 1, plain_colmac(c.P1s, pl.dA, ncol, c.Xq, nv, c.Up, pl.S1s), c.st));
    TNSLQ_HIP(launch_sum_transpose_ups(c.Up, pl.S1s, pl.K, pl.nB, pl.nE, c.U2, c.st));
    if (e1) TNSLQ_HIP(hipEventRecord(e1, c.st));
    double2 *Yt = (double2 *)c.Ypart;
    TNSLQ_HIP(launch_colmac(pl.dtype, 0, plain_colmac(c.P2s, ncol, pl.dA, c.U2, nv, Yt, pl.S2s), c.st));
    TNSLQ_HIP(launch_sum_transpose_y(Yt, pl.S2s, pl.K, pl.dA, pl.nB, c.Ym, c.st));
    if (e2) TNSLQ_HIP(hipEventRecord(e2, c.st));
    c.n_launch++;
    return TNSLQ_OK;
}

// Both contractions for probes [k0, k0 + kcur): Xt -> Ups -> Ypart.
int contract_chunk(Ctx &c, int k0, int kcur, hipEvent_t e1, hipEvent_t e2) {
    const Plan &pl = c.pl;
    // contraction 1: Ups[(k, b)][(c, b')] = sum_a' conj psi[a', b, c] Xt[(k, b')][a'];
    // output (i, j) = ((b, c), (k, b')) -> row k d_B + b, index c d_B + b'
    GemmDesc g1{};
    g1.A = c.Pbea;
    g1.B = (const char *)c.Xt + (size_t)((int64_t)k0 * pl.dB / BRICK_ROWS) * brick_block_bytes(pl.prec, pl.nst1);
    g1.C = c.Ups;
    g1.M = pl.dB * pl.dE;
    g1.N = (int64_t)kcur * pl.dB;
    g1.Kr = pl.dA;
    g1.nst = pl.nst1;
    g1.S = 1;
    g1.out_mode = 0;
    g1.cnb_log2 = pl.nB;
    g1.cni_log2 = pl.nE;
    g1.crs = pl.dB;
    g1.c_nst = pl.nst2;
    const int64_t u1n = (int64_t)kcur * pl.dB * pl.dE * pl.dB;
    if (pl.S1 > 1) {
        // split along a': partials at s * split + k (d_B d_E d_B) + (b d_E + c) d_B + b'
        g1.C = c.U1part;
        g1.S = pl.S1;
        g1.out_mode = 1;
        g1.ldc = pl.dB;
        g1.cbs = pl.dB * pl.dE * pl.dB;
        g1.c_split = (int64_t)pl.kc * pl.dB * pl.dE * pl.dB;
    }
    // contraction 2: Y[k][a][b] = sum_(c, b') psi[a, c, b'] Ups[(k, b)][(c, b')],
    // split-K partials at s * kc d_A d_B + k d_A d_B + a d_B + b
    GemmDesc g2{};
    g2.A = c.Paeb;
    g2.B = c.Ups;
    g2.C = c.Ypart;
    g2.M = pl.dA;
    g2.N = (int64_t)kcur * pl.dB;
    g2.Kr = pl.dE * pl.dB;
    g2.nst = pl.nst2;
    g2.S = pl.S;
    g2.out_mode = 1;
    g2.cnb_log2 = pl.nB;
    g2.cni_log2 = 0;
    g2.ldc = pl.dB;
    g2.cbs = pl.dAB;
    g2.c_split = (int64_t)pl.kc * pl.dAB;
    TNSLQ_HIP(launch_gemm(pl.prec, g1, c.st));
    if (pl.S1 > 1)
        TNSLQ_HIP(launch_partials_to_bricks(pl.prec, c.U1part, pl.S1, g1.c_split, u1n, pl.nB, pl.nE, c.Ups, pl.nst2,
                                            c.st));
    if (e1) TNSLQ_HIP(hipEventRecord(e1, c.st));
    TNSLQ_HIP(launch_gemm(pl.prec, g2, c.st));
    if (e2) TNSLQ_HIP(hipEventRecord(e2, c.st));
    c.n_launch++;
    return TNSLQ_OK;
}

// Intermediary (iii): Y[k][i] = sum_l rho^{T_B}[i][l] Xt[k][l] for all K
// probes, split-K partials at s K n + k n + i.
int explicit_matvec(Ctx &c, hipEvent_t e1, hipEvent_t e2) {
    const Plan &pl = c.pl;
    const int64_t n = pl.dAB;
    if (e1) TNSLQ_HIP(hipEventRecord(e1, c.st));
    GemmDesc g{};
    g.A = c.rho;
    g.B = c.Xt;
    g.C = c.Ypart;
    g.M = n;
    g.N = pl.K;
    g.Kr = n;
    g.nst = pl.nst_rho;
    g.S = pl.S;
    g.out_mode = 1;
    g.cnb_log2 = 0;
    g.cni_log2 = 0;
    g.ldc = 1;
    g.cbs = n;
    g.c_split = (int64_t)pl.K * n;
    TNSLQ_HIP(launch_gemm(pl.prec, g, c.st));
    if (e2) TNSLQ_HIP(hipEventRecord(e2, c.st));
    c.n_launch++;
    return TNSLQ_OK;
}

// rho^{T_B} of the two-block state psi[a][b][(u', v)] = sum_m P[a][u'][m]
// Q[b][m][v] (Sec. VI) applied to probes [k0, k0 + kcur) without forming psi:
//   Z1[k][(u', m')][b']     = sum_a' conj P[a'][(u', m')] X[k][a'][b']
//   Z2[k][(u', m')][(m, v)] = sum_b' Z1[k][(u', m')][b'] Q[b'][(m, v)]
//   Z2p[k][(u', m)][(m', v)]  (axes m and m' exchanged: the product writes
//                            its outputs there directly)
//   Z3[k][a][(m', v)]       = sum_(u', m) P[a][(u', m)] Z2p[k][(u', m)][(m', v)]
//   Y[k][a][b]              = sum_(m', v) Z3[k][a][(m', v)] conj Q[b][(m', v)]
// i.e. Y[a][b] = sum_{a', b', e} psi[a][b'][e] conj psi[a'][b][e] X[a'][b'].
int mps_matvec(Ctx &c, const double2 *x, int kcur, hipEvent_t e1, hipEvent_t e2) {
    const Plan &pl = c.pl;
    const MpsFactors &f = c.mf;
    const int64_t n = pl.dAB, UpM = f.Up * f.M, MV = f.M * f.V;
    const int kA = (int)f.kA, kB = (int)f.kB;
    auto chain = [&](auto *P, auto *Q, auto *X, auto *Z1, auto *Z2, auto *Z2p, auto *Z3, auto *Y) -> int {
        TNSLQ_HIP(launch_zgemm(2, 0, P, X, Z1, (int)UpM, kB, kA, UpM, kB, kB, kcur, 0, n, UpM * kB, c.st));
        if (UpM <= 65535 * 64) {
            // Z2 written straight into the exchanged order Z2p
            TNSLQ_HIP(launch_zgemm_xc(Z1, Q, Z2p, (int)UpM, (int)MV, kB, kB, MV, kcur, UpM * kB, 0, UpM * MV, f.M,
                                      f.V, c.st));
            if (e1) TNSLQ_HIP(hipEventRecord(e1, c.st));
        } else {
            TNSLQ_HIP(launch_zgemm(0, 0, Z1, Q, Z2, (int)UpM, (int)MV, kB, kB, MV, MV, kcur, UpM * kB, 0, UpM * MV,
                                   c.st));
            if (e1) TNSLQ_HIP(hipEventRecord(e1, c.st));
            TNSLQ_HIP(launch_swap01(Z2, (int64_t)kcur * f.Up, f.M, f.M, f.V, Z2p, c.st));
        }
        TNSLQ_HIP(launch_zgemm(0, 0, P, Z2p, Z3, kA, (int)MV, (int)UpM, UpM, MV, MV, kcur, 0, UpM * MV, kA * MV,
                               c.st));
        // split s of the reduction at Y + s kc n (passA sums the splits)
        TNSLQ_HIP(launch_zgemm(0, 2, Z3, Q, Y, kA, kB, (int)MV, MV, MV, kB, kcur, kA * MV, 0, n, c.st, 0, pl.S,
                               (int64_t)pl.kc * n));
        return TNSLQ_OK;
    };
    int rc;
    if (pl.prec == TNSLQ_FP32) {
        TNSLQ_HIP(launch_to_c64(x, (int64_t)kcur * n, c.X32, c.st));
        rc = chain((const float2 *)c.P32, (const float2 *)c.Q32, (const float2 *)c.X32, (float2 *)c.Z1,
                   (float2 *)c.Z2, (float2 *)c.Z2p, (float2 *)c.Z3, (float2 *)c.Ypart);
    } else {
        rc = chain((const double2 *)f.P, f.Q, x, c.Z1, c.Z2, c.Z2p, c.Z3, (double2 *)c.Ypart);
    }
    if (rc) return rc;
    if (e2) TNSLQ_HIP(hipEventRecord(e2, c.st));
    c.n_launch++;
    return TNSLQ_OK;
}

// The network form's matvec for kcur probes (x: [k][a'][b'], kA x kB each):
//   T1[k][(u', m')][b']    = sum_a' conj R_A[a'][(u', m')] X[k][a'][b']
//   T2[k][(u', m')][(n, v)] = sum_b' T1 R_B[b'][(n, v)]
//   T3[k][m][n'][u'][v]    = sum_{m', n} E_W[m][n][m'][n'] T2[k][u'][m'][n][v]
//                            (adjacent blocks: T2 regrouped, n = m, n' = m')
//   T4[k][u][v'][m][n']    = sum_{v, u'} E_Z[v][u][v'][u'] T3[k][m][n'][u'][v]
//                            (open chain: T3 regrouped, u' = u, v' = v)
//   T5[k][a][(n', v')]     = sum_{u, m} R_A[a][(u, m)] T4[k][u][v'][m][n']
//   Y[k][a][b]             = sum_{n', v'} T5[k][a][(n', v')] conj R_B[b][(n', v')]
// (the last in reduction splits at Ypart, as for the factors).  Each product
// is batched over the chunk; the regroupings are axis permutations.
int net_matvec(Ctx &c, const double2 *x, int kcur, hipEvent_t e1, hipEvent_t e2) {
    const Plan &pl = c.pl;
    const int64_t n = pl.dAB, U = pl.nU, M = pl.nM, N = pl.nN, V = pl.nV, UM = U * M, NV = N * V, MN = M * N,
                  UV = U * V, big = UM * NV;
    const int kA = (int)pl.dA, kB = (int)pl.dB;
    const NetBufs nb = net_bufs(pl);
    char *base = c.ws + pl.off_net;
    auto chain = [&](auto *RA, auto *RB, auto *EWp, auto *EZp, auto *X, auto *T1, auto *Ta, auto *Tb, auto *T5,
                     auto *Y) -> int {
        TNSLQ_HIP(launch_zgemm(2, 0, RA, X, T1, (int)UM, kB, kA, UM, kB, kB, kcur, 0, n, UM * kB, c.st));
        TNSLQ_HIP(launch_zgemm(0, 0, T1, RB, Ta, (int)UM, (int)NV, kB, kB, NV, NV, kcur, UM * kB, 0, big, c.st));
        if (e1) TNSLQ_HIP(hipEventRecord(e1, c.st));
        auto *T3 = Ta;   // [m][n'][u'][v]
        if (pl.ngap) {
            const int64_t d[4] = {U, M, N, V};
            const int perm[4] = {1, 2, 0, 3};   // [m'][n][u'][v]
            TNSLQ_HIP(launch_permute4(Ta, d, perm, Tb, c.st, kcur));
            TNSLQ_HIP(launch_zgemm(0, 0, EWp, Tb, Ta, (int)MN, (int)UV, (int)MN, MN, UV, UV, kcur, 0, big, big, c.st));
        } else {
            const int64_t d[4] = {U, M, M, V};
            const int perm[4] = {2, 1, 0, 3};
            TNSLQ_HIP(launch_permute4(Ta, d, perm, Tb, c.st, kcur));
            T3 = Tb;
        }
        auto *other = T3 == Ta ? Tb : Ta;
        auto *T4p = other;   // [u][m][n'][v']
        if (pl.nring) {
            const int64_t d3[4] = {M, N, U, V};
            const int perm3[4] = {3, 2, 0, 1};   // [v][u'][m][n']
            TNSLQ_HIP(launch_permute4(T3, d3, perm3, other, c.st, kcur));
            TNSLQ_HIP(launch_zgemm(0, 0, EZp, other, T3, (int)UV, (int)MN, (int)UV, UV, MN, MN, kcur, 0, big, big,
                                   c.st));   // T4[u][v'][m][n']
            const int64_t d4[4] = {U, V, M, N};
            const int perm4[4] = {0, 2, 3, 1};
            TNSLQ_HIP(launch_permute4(T3, d4, perm4, other, c.st, kcur));
        } else {
            const int64_t d3[4] = {M, N, U, V};
            const int perm3[4] = {2, 0, 1, 3};
            TNSLQ_HIP(launch_permute4(T3, d3, perm3, other, c.st, kcur));
        }
        TNSLQ_HIP(launch_zgemm(0, 0, RA, T4p, T5, kA, (int)NV, (int)UM, UM, NV, NV, kcur, 0, big, kA * NV, c.st));
        TNSLQ_HIP(launch_zgemm(0, 2, T5, RB, Y, kA, kB, (int)NV, NV, NV, kB, kcur, kA * NV, 0, n, c.st, 0, pl.S,
                               (int64_t)pl.kc * n));
        return TNSLQ_OK;
    };
    int rc;
    if (pl.prec == TNSLQ_FP32) {
        TNSLQ_HIP(launch_to_c64(x, (int64_t)kcur * n, c.X32, c.st));
        rc = chain((const float2 *)c.P32, (const float2 *)c.Q32, (const float2 *)(base + nb.ew32),
                   (const float2 *)(base + nb.ez32), (const float2 *)c.X32, (float2 *)c.Z1, (float2 *)c.Z2,
                   (float2 *)c.Z2p, (float2 *)c.Z3, (float2 *)c.Ypart);
    } else {
        rc = chain((const double2 *)c.mf.RA, c.mf.RB, (const double2 *)(base + nb.ewp),
                   (const double2 *)(base + nb.ezp), x, c.Z1, c.Z2, c.Z2p, c.Z3, (double2 *)c.Ypart);
    }
    if (rc) return rc;
    if (e2) TNSLQ_HIP(hipEventRecord(e2, c.st));
    c.n_launch++;
    return TNSLQ_OK;
}

// Events of one Lanczos step: mv0, then per probe chunk (after contraction 1,
// after contraction 2, after the merge), then mv1 (matvec done), lz1.
struct StepEvents {
    std::vector<hipEvent_t> e;
    int nchunk = 0;
    hipEvent_t mv0() const { return e[0]; }
    hipEvent_t c1(int ch) const { return e[1 + 3 * ch]; }
    hipEvent_t c2(int ch) const { return e[2 + 3 * ch]; }
    hipEvent_t pa(int ch) const { return e[3 + 3 * ch]; }
    hipEvent_t mv1() const { return e[1 + 3 * nchunk]; }
    hipEvent_t lz1() const { return e[2 + 3 * nchunk]; }
};

int lanczos_step(Ctx &c, int j, StepEvents *se) {
    const Plan &pl = c.pl;
    const int64_t n = pl.dAB;
    const int64_t slot = (int64_t)pl.K * n;
    auto slot_of = [&](int jj) { return pl.reorth ? jj : jj % 3; };   // q_{jj+1} lives in slot slot_of(jj)
    double2 *q_cur = c.Q + slot_of(j - 1) * slot;
    double2 *q_prev = j > 1 ? c.Q + slot_of(j - 2) * slot : q_cur;
    double2 *q_next = c.Q + slot_of(j) * slot;
    const int accfp64 = pl.prec == TNSLQ_FP64 || pl.stream;
    int rc;
    TNSLQ_HIP(hipEventRecord(se->mv0(), c.st));
    for (int k0 = 0, ch = 0; k0 < pl.K; k0 += pl.kc, ++ch) {
        const int kcur = std::min(pl.kc, pl.K - k0);
        if (pl.mpsf) {
            if ((rc = (pl.mnet ? net_matvec : mps_matvec)(c, q_cur + (int64_t)k0 * n, kcur, se->c1(ch), se->c2(ch))))
                return rc;
        } else if (pl.expl) {
            if ((rc = explicit_matvec(c, se->c1(ch), se->c2(ch)))) return rc;
        } else if (pl.stream) {
            if ((rc = stream_contract(c, q_cur, se->c1(ch), se->c2(ch)))) return rc;
        } else if ((rc = contract_chunk(c, k0, kcur, se->c1(ch), se->c2(ch)))) {
            return rc;
        }
        // the streaming passes leave Y already summed over their splits
        TNSLQ_HIP(launch_passA(accfp64, c.z, pl.stream && !pl.fused ? (const void *)c.Ym : c.Ypart,
                               pl.stream && !pl.fused ? 1 : pl.S,
                               (int64_t)pl.kc * n, k0, kcur, q_prev, q_cur, c.w, c.alpha, c.beta, j, c.dotpart,
                               c.st));
        TNSLQ_HIP(hipEventRecord(se->pa(ch), c.st));
    }
    TNSLQ_HIP(hipEventRecord(se->mv1(), c.st));
    TNSLQ_HIP(launch_passB(c.z, c.dotpart, q_cur, c.w, c.alpha, c.beta, j, c.nrmpart, pl.reorth ? 0 : 1, c.st));
    if (pl.reorth)
        TNSLQ_HIP(launch_reorth(c.z, c.Q, j, slot, c.w, c.hpart, c.h, c.alpha, c.beta, j, c.nrmpart, c.st));
    TNSLQ_HIP(launch_passC(pl.prec, c.z, c.nrmpart, c.w, q_next, pl.stream ? nullptr : c.Xt, pl.nst1, c.alpha,
                           c.beta, j, c.st));
    TNSLQ_HIP(hipEventRecord(se->lz1(), c.st));
    return TNSLQ_OK;
}

int slq_setup(Ctx &c, const void *psi, uint64_t seed, uint64_t offset) {
    const Plan &pl = c.pl;
    int rc;
    if ((rc = do_layout(c, psi))) return rc;
    TNSLQ_HIP(launch_zero(c.alpha, (size_t)pl.K * pl.m * 8, c.st));
    TNSLQ_HIP(launch_zero(c.beta, (size_t)pl.K * (pl.m + 1) * 8, c.st));
    TNSLQ_HIP(launch_zero(c.F, (size_t)pl.K * pl.m * 8, c.st));
    TNSLQ_HIP(launch_probe_init(pl.prec, c.z, seed, offset, pl.swapped, c.Q, pl.stream ? nullptr : c.Xt, pl.nst1,
                                c.alpha, c.beta, c.st));
    return TNSLQ_OK;
}

// Quadrature for steps [jlo, jhi] and the statistics of step `jstat`.
int quad_stats(Ctx &c, int jdone, int jlo, int jhi, int jstat, double *G) {
    const Plan &pl = c.pl;
    TNSLQ_HIP(launch_steps(c.alpha, c.beta, pl.K, pl.m, jdone, c.steps, c.st));
    TNSLQ_HIP(launch_quadrature(c.alpha, c.beta, c.steps, pl.K, pl.m, jlo, jhi, TNSLQ_F_ABS, c.F, c.st));
    TNSLQ_HIP(launch_stats(c.beta, c.F, pl.K, pl.m, jstat, G, c.stats, c.st));
    return TNSLQ_OK;
}

float elapsed(hipEvent_t a, hipEvent_t b) {
    float ms = 0.f;
    if (a && b && hipEventElapsedTime(&ms, a, b) == hipSuccess) return ms;
    return 0.f;
}

void zero_result(tnslq_result *res) {
    memset(res, 0, sizeof *res);
}

// Trivial partitions (empty A or B): rho^{T_B} then has the spectrum of a
// density matrix, so the trace norm is 1 and E = 0 exactly.
int trivial(const tnslq_options *opt, tnslq_result *res, double *G, double *alpha, double *beta, double *F,
            int *steps) {
    zero_result(res);
    res->trace_norm = 1.0;
    const int K = opt->n_probes, m = opt->n_steps;
    res->n_probes_used = K;
    if (G) std::fill(G, G + K, 1.0);
    if (alpha) std::fill(alpha, alpha + (size_t)K * m, 0.0);
    if (beta) std::fill(beta, beta + (size_t)K * (m + 1), 0.0);
    if (F) std::fill(F, F + (size_t)K * m, 1.0);
    if (steps) std::fill(steps, steps + K, 0);
    return TNSLQ_OK;
}

// The estimate needs a normalised state (Tr rho_AB = 1, Eq. 1); psi is
// checked, not silently renormalised: its non-finite amplitudes and its
// squared norm are read back once before the Lanczos steps.  Synchronises.
int check_state(int dtype, const void *psi, int64_t D, double *scratch, hipStream_t st) {
    TNSLQ_HIP(launch_state_check(dtype, psi, D, scratch, st));
    double h[2];
    TNSLQ_HIP(hipMemcpyAsync(h, scratch + 2 * STATE_CHECK_BLOCKS, sizeof h, hipMemcpyDeviceToHost, st));
    TNSLQ_HIP(hipStreamSynchronize(st));
    if (h[1] > 0.0) return fail(TNSLQ_E_NONFINITE, "psi holds %.0f non-finite amplitudes", h[1]);
    const double tol = dtype == TNSLQ_C128 ? TNSLQ_NORM_TOL_C128 : TNSLQ_NORM_TOL_C64;
    if (!(std::fabs(h[0] - 1.0) <= tol))
        return fail(TNSLQ_E_STATE, "psi is not normalised: ||psi||^2 = %.10g (tolerance %g)", h[0], tol);
    return TNSLQ_OK;
}

int check_options(const tnslq_options *opt) {
    if (!opt) return fail(TNSLQ_E_ARG, "options is NULL");
    if (opt->n_probes < 1) return fail(TNSLQ_E_ARG, "n_probes must be >= 1");
    if (opt->n_steps < 1 || opt->n_steps > TNSLQ_MAX_STEPS)
        return fail(TNSLQ_E_ARG, "n_steps %d outside [1, %d]", opt->n_steps, TNSLQ_MAX_STEPS);
    if (opt->reorth != 0 && opt->reorth != 1) return fail(TNSLQ_E_ARG, "reorth must be 0 or 1");
    if (!(opt->stop_tol >= 0.0)) return fail(TNSLQ_E_ARG, "stop_tol must be >= 0");
    if (opt->stop_rule != TNSLQ_STOP_DIFF && opt->stop_rule != TNSLQ_STOP_FIT)
        return fail(TNSLQ_E_ARG, "stop_rule %d unknown", opt->stop_rule);
    if (opt->operator_form < TNSLQ_OPERATOR_AUTO || opt->operator_form > TNSLQ_OPERATOR_LAZY_TWO_PASS)
        return fail(TNSLQ_E_ARG, "operator_form %d unknown", opt->operator_form);
    if (opt->max_probes < 0) return fail(TNSLQ_E_ARG, "max_probes must be >= 0");
    if (opt->chunk_probes < 0) return fail(TNSLQ_E_ARG, "chunk_probes must be >= 0");
    if (opt->max_probes > opt->n_probes && (opt->stop_rule != TNSLQ_STOP_FIT || !(opt->stop_tol > 0.0)))
        return fail(TNSLQ_E_ARG, "the loop over probes (max_probes > n_probes) needs the fit rule and stop_tol > 0");
    if (opt->stop_rule == TNSLQ_STOP_FIT && opt->n_steps < TNSLQ_FIT_MIN_POINTS + 1)
        return fail(TNSLQ_E_ARG, "the fit rule needs n_steps >= %d", TNSLQ_FIT_MIN_POINTS + 1);
    return check_prec(opt->precision);
}

struct Timer {
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
    double ms() const {
        return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
};

// Shared body of tnslq_logneg and tnslq_logneg_surrogate.
struct Run {
    Ctx c;
    std::vector<StepEvents> se;
    hipEvent_t e_start = nullptr, e_layout = nullptr;
    int jdone = 0;
    int rule = TNSLQ_STOP_DIFF;
    double lanczos_err = 0.0;   // of the last stop check
    bool target = false;        // the last run_steps had a target (stop_tol > 0)
    bool met = false;           // and stopped because it was met
};

int run_start(Run &r, const tnslq_options *opt, const void *psi, void *ws, size_t ws_bytes, void *stream);

int run_begin(Run &r, int dtype, const tnslq_partition *part, const tnslq_options *opt, const void *psi, void *ws,
              size_t ws_bytes, void *stream) {
    int rc;
    if ((rc = make_plan(dtype, part, opt->n_probes, opt->n_steps, opt->reorth, opt->precision, 1,
                         opt->operator_form, r.c.pl, opt->chunk_probes)))
        return rc;
    return run_start(r, opt, psi, ws, ws_bytes, stream);
}

// Bind the workspace to a planned run, regroup psi and start the probes.
int run_start(Run &r, const tnslq_options *opt, const void *psi, void *ws, size_t ws_bytes, void *stream) {
    int rc;
    if (!psi) return fail(TNSLQ_E_ARG, "psi is NULL");
    if (!ws) return fail(TNSLQ_E_ARG, "workspace is NULL");
    if ((uintptr_t)ws % ALIGN) return fail(TNSLQ_E_ARG, "workspace not 256-byte aligned");
    if (ws_bytes < r.c.pl.total)
        return fail(TNSLQ_E_WORKSPACE, "workspace %zu bytes, need %zu", ws_bytes, r.c.pl.total);
    bind(r.c, ws, (hipStream_t)stream);
    r.rule = opt->stop_rule;
    r.e_start = r.c.event();
    r.e_layout = r.c.event();
    r.se.resize(opt->n_steps + 1);
    const int nchunk = (r.c.pl.K + r.c.pl.kc - 1) / r.c.pl.kc;
    for (auto &s : r.se) {
        s.nchunk = nchunk;
        s.e.resize(3 + 3 * nchunk);
        for (auto &e : s.e)
            if (!(e = r.c.event())) return fail(TNSLQ_E_DEVICE, "hipEventCreate failed");
    }
    TNSLQ_HIP(hipEventRecord(r.e_start, r.c.st));
    if (!r.c.pl.mpsf && (rc = check_state(r.c.pl.dtype, psi, r.c.pl.D, (double *)(r.c.ws + r.c.pl.off_chk), r.c.st)))
        return rc;
    roctxRangePush("tnslq layout");
    rc = slq_setup(r.c, psi, opt->seed, opt->probe_offset);
    roctxRangePop();
    if (rc) return rc;
    TNSLQ_HIP(hipEventRecord(r.e_layout, r.c.st));
    return TNSLQ_OK;
}

// Fitted estimate of every probe after step j (exponential fit, Sec. III):
// quadrature of the window's steps, the fits and their block statistics.
int fit_step(Run &r, int j, double *G) {
    Ctx &c = r.c;
    const int lo = std::max(2, j - TNSLQ_FIT_WINDOW + 1);
    TNSLQ_HIP(launch_steps(c.alpha, c.beta, c.pl.K, c.pl.m, j, c.steps, c.st));
    TNSLQ_HIP(launch_quadrature(c.alpha, c.beta, c.steps, c.pl.K, c.pl.m, lo, j, TNSLQ_F_ABS, c.F, c.st));
    TNSLQ_HIP(launch_fit(c.alpha, c.beta, c.F, c.pl.K, c.pl.m, j, c.finf, c.fsig, G, c.fitout, c.st));
    return TNSLQ_OK;
}

// Steps jdone+1 .. jmax; with stop_tol > 0 stops at the first step meeting the
// precision target under the run's stopping rule (for the fit rule with
// lanczos_only, on the Lanczos part of the error alone).
int run_steps(Run &r, int jmax, double stop_tol, bool lanczos_only = false) {
    int rc;
    r.target = stop_tol > 0.0;
    r.met = false;
    for (int j = r.jdone + 1; j <= jmax; ++j) {
        roctxRangePush("tnslq lanczos step");
        rc = lanczos_step(r.c, j, &r.se[j]);
        roctxRangePop();
        if (rc) return rc;
        r.jdone = j;
        if (stop_tol <= 0.0) continue;
        if (r.rule == TNSLQ_STOP_FIT && j >= TNSLQ_FIT_MIN_POINTS + 1) {
            if ((rc = fit_step(r, j, nullptr))) return rc;
            double o[6];
            TNSLQ_HIP(hipMemcpyAsync(o, r.c.fitout, sizeof o, hipMemcpyDeviceToHost, r.c.st));
            TNSLQ_HIP(hipStreamSynchronize(r.c.st));
            // lanczos_only: the block's Lanczos error alone, eps_L / (T ln 2)
            const double err = lanczos_only ? o[2] / (o[0] * std::log(2.0)) : o[4];
            if (std::isfinite(o[3]) && std::isfinite(err) && err <= stop_tol * std::max(std::fabs(o[3]), 1.0)) {
                r.met = true;
                break;
            }
        } else if (r.rule == TNSLQ_STOP_DIFF && j >= 6) {
            if ((rc = quad_stats(r.c, j, j - 5, j, j - 5, nullptr))) return rc;
            TNSLQ_HIP(launch_stats(r.c.beta, r.c.F, r.c.pl.K, r.c.pl.m, j, nullptr, r.c.stats, r.c.st));
            double s[8];
            TNSLQ_HIP(hipMemcpyAsync(s, r.c.stats + (size_t)(j - 6) * 4, 4 * sizeof(double), hipMemcpyDeviceToHost,
                                     r.c.st));
            TNSLQ_HIP(hipMemcpyAsync(s + 4, r.c.stats + (size_t)(j - 1) * 4, 4 * sizeof(double),
                                     hipMemcpyDeviceToHost, r.c.st));
            TNSLQ_HIP(hipStreamSynchronize(r.c.st));
            const double e_now = s[6], de = s[7], e_old = s[2];
            const double dl = e_now - e_old;
            const double err = std::sqrt((std::isnan(de) ? 0.0 : de * de) + dl * dl);
            if (std::isfinite(e_now) && err <= stop_tol * std::max(std::fabs(e_now), 1.0)) {
                r.met = true;
                break;
            }
        }
    }
    return TNSLQ_OK;
}

int run_finish(Run &r, tnslq_result *res, double *G, double *alpha, double *beta, double *F, int *steps,
               const Timer &tm) {
    Ctx &c = r.c;
    const Plan &pl = c.pl;
    int rc;
    const bool fit = r.rule == TNSLQ_STOP_FIT && r.jdone >= TNSLQ_FIT_MIN_POINTS + 1;
    // A fit-rule run that had a target and ran out of steps without meeting
    // it reports the plain estimate of its last step (the fitted limit of a
    // trajectory that has not settled can be far off), with the fit's
    // Lanczos error as the measure of how far it is from converged.
    const bool plain = !fit || (r.target && !r.met);
    // quadrature of every step and the plain statistics of each step (G at the
    // last step unless the fit supplies it)
    if ((rc = quad_stats(c, r.jdone, 1, r.jdone, r.jdone, plain ? c.G : nullptr))) return rc;
    if (fit && (rc = fit_step(r, r.jdone, plain ? nullptr : c.G))) return rc;
    double s[4], o[6], e_old = std::nan("");
    TNSLQ_HIP(hipMemcpyAsync(s, c.stats + (size_t)(r.jdone - 1) * 4, sizeof s, hipMemcpyDeviceToHost, c.st));
    if (fit) TNSLQ_HIP(hipMemcpyAsync(o, c.fitout, sizeof o, hipMemcpyDeviceToHost, c.st));
    if (!fit && r.jdone >= 6) {
        TNSLQ_HIP(launch_stats(c.beta, c.F, pl.K, pl.m, r.jdone - 5, nullptr, c.stats, c.st));
        TNSLQ_HIP(hipMemcpyAsync(&e_old, c.stats + (size_t)(r.jdone - 6) * 4 + 2, sizeof(double),
                                 hipMemcpyDeviceToHost, c.st));
    }
    std::vector<int> hsteps(pl.K);
    TNSLQ_HIP(hipMemcpyAsync(hsteps.data(), c.steps, sizeof(int) * pl.K, hipMemcpyDeviceToHost, c.st));
    if (G) TNSLQ_HIP(hipMemcpyAsync(G, c.G, sizeof(double) * pl.K, hipMemcpyDeviceToHost, c.st));
    if (alpha) TNSLQ_HIP(hipMemcpyAsync(alpha, c.alpha, sizeof(double) * pl.K * pl.m, hipMemcpyDeviceToHost, c.st));
    if (beta)
        TNSLQ_HIP(hipMemcpyAsync(beta, c.beta, sizeof(double) * pl.K * (pl.m + 1), hipMemcpyDeviceToHost, c.st));
    if (F) TNSLQ_HIP(hipMemcpyAsync(F, c.F, sizeof(double) * pl.K * pl.m, hipMemcpyDeviceToHost, c.st));
    TNSLQ_HIP(hipStreamSynchronize(c.st));
    if (steps) std::copy(hsteps.begin(), hsteps.end(), steps);
    zero_result(res);
    if (!plain) {
        const double ln2 = std::log(2.0);
        res->trace_norm = o[0];
        res->trace_norm_se = pl.K > 1 ? o[1] : std::nan("");
        res->logneg = o[3];
        res->logneg_se = o[5];
        res->lanczos_err = o[2] / (o[0] * ln2);
    } else {
        res->trace_norm = s[0];
        res->trace_norm_se = s[1];
        res->logneg = s[2];
        res->logneg_se = s[3];
        if (fit)
            res->lanczos_err = o[2] / (o[0] * std::log(2.0));
        else
            res->lanczos_err = r.jdone >= 6 ? std::fabs(s[2] - e_old) : std::nan("");
    }
    res->steps_done = r.jdone;
    res->steps_min = *std::min_element(hsteps.begin(), hsteps.end());
    res->swapped_ab = pl.swapped;
    res->streamed = pl.stream ? (pl.fused ? 2 : 1) : 0;
    res->explicit_operator = pl.expl;
    res->mps_matvec = pl.mpsf ? (pl.mnet ? TNSLQ_MPS_MATVEC_NETWORK : TNSLQ_MPS_MATVEC_FACTORS) : 0;
    res->n_probes_used = pl.K;
    res->n_matvecs = r.jdone;
    res->n_contract_launches = c.n_launch;
    res->t_layout_ms = elapsed(r.e_start, r.e_layout);
    for (int j = 1; j <= r.jdone; ++j) {
        const StepEvents &e = r.se[j];
        res->t_matvec_ms += elapsed(e.mv0(), e.mv1());
        for (int ch = 0; ch < e.nchunk; ++ch) {
            res->t_contract1_ms += elapsed(ch == 0 ? e.mv0() : e.pa(ch - 1), e.c1(ch));
            res->t_contract2_ms += elapsed(e.c1(ch), e.c2(ch));
        }
        res->t_lanczos_ms += elapsed(e.mv1(), e.lz1());
    }
    res->t_total_ms = tm.ms();
    if (!std::isfinite(res->logneg))
        return fail(TNSLQ_E_NONFINITE, "estimate is not finite (trace norm %g)", res->trace_norm);
    return TNSLQ_OK;
}


// ------------------------------------------------------------ spectral sums
// Tr f(rho_S) for f = -x log2 x or x^2 by Algorithm 1 on the reduced density
// matrix of the smaller side, applied as two passes over psi (entropy.hip).
struct SPlan {
    int L = 0, dtype = TNSLQ_C64, fn = TNSLQ_F_ENTROPY;
    int n_side = 0, n_rest = 0, complement = 0;
    int side[TNSLQ_MAX_QUBITS], rest[TNSLQ_MAX_QUBITS];
    int64_t d = 1, dR = 1, D = 1;
    int K = 1, m = 1, reorth = 0;
    int S1 = 1, S2 = 1, nblk = 1, nQ = 3;
    size_t off_P1 = 0, off_P2 = 0, off_Zp = 0, off_Z = 0, off_Yp = 0, off_Q = 0, off_w = 0, off_alpha = 0, off_beta = 0;
    size_t off_F = 0, off_G = 0, off_stats = 0, off_red = 0, off_h = 0, off_steps = 0, off_chk = 0, total = 0;
};

int check_subsystem(int L, const int *s, int n_s) {
    if (L < 1 || L > TNSLQ_MAX_QUBITS) return fail(TNSLQ_E_PARTITION, "n_qubits %d outside [1, %d]", L, TNSLQ_MAX_QUBITS);
    if (n_s < 0 || n_s > L) return fail(TNSLQ_E_PARTITION, "subsystem size %d outside [0, %d]", n_s, L);
    if (n_s > 0 && !s) return fail(TNSLQ_E_ARG, "qubit list is NULL");
    std::vector<int> seen(L, 0);
    for (int i = 0; i < n_s; ++i) {
        if (s[i] < 0 || s[i] >= L) return fail(TNSLQ_E_PARTITION, "qubit %d out of range", s[i]);
        if (seen[s[i]]) return fail(TNSLQ_E_PARTITION, "qubit %d repeated", s[i]);
        seen[s[i]] = 1;
    }
    return TNSLQ_OK;
}

int check_spectral_options(const tnslq_options *opt, int fn) {
    int rc;
    if ((rc = check_options(opt))) return rc;
    if (fn != TNSLQ_F_ENTROPY && fn != TNSLQ_F_PURITY) return fail(TNSLQ_E_ARG, "function %d unknown", fn);
    if (opt->precision != TNSLQ_FP64) return fail(TNSLQ_E_ARG, "spectral sums compute in FP64 only");
    if (opt->stop_tol != 0.0) return fail(TNSLQ_E_ARG, "spectral sums run a fixed number of steps (stop_tol 0)");
    return TNSLQ_OK;
}

int make_splan(int dtype, int L, const int *s, int n_s, const tnslq_options *opt, int fn, SPlan &sp) {
    int rc;
    if ((rc = check_dtype(dtype)) || (rc = check_subsystem(L, s, n_s)) || (rc = check_spectral_options(opt, fn)))
        return rc;
    sp = SPlan();
    sp.L = L;
    sp.dtype = dtype;
    sp.fn = fn;
    std::vector<int> in_s(L, 0), comp;
    for (int i = 0; i < n_s; ++i) in_s[s[i]] = 1;
    for (int q = 0; q < L; ++q)
        if (!in_s[q]) comp.push_back(q);
    sp.complement = n_s > L - n_s;
    const int *side = sp.complement ? comp.data() : s;
    const int *rest = sp.complement ? s : comp.data();
    sp.n_side = sp.complement ? L - n_s : n_s;
    sp.n_rest = L - sp.n_side;
    for (int i = 0; i < sp.n_side; ++i) sp.side[i] = side[i];
    for (int i = 0; i < sp.n_rest; ++i) sp.rest[i] = rest[i];
    sp.d = int64_t(1) << sp.n_side;
    sp.dR = int64_t(1) << sp.n_rest;
    sp.D = int64_t(1) << L;
    sp.K = opt->n_probes;
    sp.m = opt->n_steps;
    sp.reorth = opt->reorth;
    // row splits of the two passes: about 2048 blocks, at least 64 rows each
    const int64_t kg = (sp.K + 7) / 8;
    const int64_t cb1 = (sp.dR + 511) / 512 * kg, cb2 = (sp.d + 511) / 512 * kg;
    while (cb1 * sp.S1 < 2048 && sp.d / (2 * sp.S1) >= 64 && sp.S1 < 1024) sp.S1 *= 2;
    while (cb2 * sp.S2 < 2048 && sp.dR / (2 * sp.S2) >= 64 && sp.S2 < 1024) sp.S2 *= 2;
    sp.nblk = reduction_blocks(sp.d, sp.K);
    sp.nQ = sp.reorth ? sp.m + 1 : 3;
    const size_t esz = dtype == TNSLQ_C128 ? 16 : 8;
    const int K = sp.K, m = sp.m;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t r = o;
        o += up(bytes);
        return r;
    };
    sp.off_P1 = take(esz * (size_t)sp.D);
    sp.off_P2 = take(esz * (size_t)sp.D);
    sp.off_Zp = take((size_t)sp.S1 * K * sp.dR * 16);
    sp.off_Z = take((size_t)K * sp.dR * 16);
    sp.off_Yp = take((size_t)sp.S2 * K * sp.d * 16);
    sp.off_Q = take((size_t)sp.nQ * K * sp.d * 16);
    sp.off_w = take((size_t)K * sp.d * 16);
    sp.off_alpha = take((size_t)K * m * 8);
    sp.off_beta = take((size_t)K * (m + 1) * 8);
    sp.off_F = take((size_t)K * m * 8);
    sp.off_G = take((size_t)K * 8);
    sp.off_stats = take((size_t)m * 4 * 8);
    sp.off_red = take((size_t)2 * K * sp.nblk * 8);
    sp.off_h = take((size_t)K * (m + 1) * sp.nblk * 16 + (size_t)K * (m + 1) * 16);
    sp.off_steps = take((size_t)K * 4);
    sp.off_chk = take(STATE_CHECK_BYTES);
    sp.total = o;
    return TNSLQ_OK;
}

void spectral_trivial(const SPlan *sp, int fn, const tnslq_options *opt, tnslq_spectral_result *res, double *G,
                      double *alpha, double *beta, double *F, int *steps) {
    memset(res, 0, sizeof *res);
    const double v = fn == TNSLQ_F_ENTROPY ? 0.0 : 1.0;
    res->value = v;
    (void)sp;
    const int K = opt->n_probes, m = opt->n_steps;
    if (G) std::fill(G, G + K, v);
    if (alpha) std::fill(alpha, alpha + (size_t)K * m, 0.0);
    if (beta) std::fill(beta, beta + (size_t)K * (m + 1), 0.0);
    if (F) std::fill(F, F + (size_t)K * m, v);
    if (steps) std::fill(steps, steps + K, 0);
}

// The whole spectral sum with a validated plan, on the caller's workspace.
int spectral_run(const SPlan &sp, const void *psi, const tnslq_options *opt, uint64_t offset, void *ws,
                 hipStream_t st, tnslq_spectral_result *res, double *Gh, double *alh, double *beh, double *Fh,
                 int *sth, const Timer &tm) {
    char *base = (char *)ws;
    void *P1 = base + sp.off_P1, *P2 = base + sp.off_P2;
    double2 *Zp = (double2 *)(base + sp.off_Zp), *Z = (double2 *)(base + sp.off_Z);
    double2 *Yp = (double2 *)(base + sp.off_Yp);
    double2 *Q = (double2 *)(base + sp.off_Q), *w = (double2 *)(base + sp.off_w);
    double *alpha = (double *)(base + sp.off_alpha), *beta = (double *)(base + sp.off_beta);
    double *F = (double *)(base + sp.off_F), *G = (double *)(base + sp.off_G);
    double *stats = (double *)(base + sp.off_stats);
    double *dotpart = (double *)(base + sp.off_red), *nrmpart = dotpart + (size_t)sp.K * sp.nblk;
    double *hpart = (double *)(base + sp.off_h);
    double2 *h = (double2 *)(base + sp.off_h + (size_t)sp.K * (sp.m + 1) * sp.nblk * 16);
    int *steps = (int *)(base + sp.off_steps);
    const LzDims z{sp.d, 1, sp.d, sp.K, sp.m, sp.nblk};
    const int64_t n = sp.d, slot = (int64_t)sp.K * n;
    std::vector<hipEvent_t> ev;
    struct Guard {
        std::vector<hipEvent_t> &e;
        ~Guard() {
            for (auto x : e) (void)hipEventDestroy(x);
        }
    } guard{ev};
    auto event = [&]() {
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) == hipSuccess) ev.push_back(e);
        return e;
    };
    hipEvent_t e0 = event(), e1 = event();
    std::vector<hipEvent_t> mv0(sp.m + 1), mv1(sp.m + 1), lz1(sp.m + 1);
    for (int j = 1; j <= sp.m; ++j) {
        mv0[j] = event();
        mv1[j] = event();
        lz1[j] = event();
    }
    if ((int)ev.size() != 2 + 3 * sp.m) return fail(TNSLQ_E_DEVICE, "hipEventCreate failed");
    int rc0;
    if ((rc0 = check_state(sp.dtype, psi, sp.D, (double *)(base + sp.off_chk), st))) return rc0;
    TNSLQ_HIP(hipEventRecord(e0, st));
    const PermDesc p1 = perm_two(sp.L, sp.side, sp.n_side, sp.rest, sp.n_rest);
    const PermDesc p2 = perm_two(sp.L, sp.rest, sp.n_rest, sp.side, sp.n_side);
    TNSLQ_HIP(launch_regroup(sp.dtype, psi, P1, sp.d, sp.dR, p1, st));
    TNSLQ_HIP(launch_regroup(sp.dtype, psi, P2, sp.dR, sp.d, p2, st));
    TNSLQ_HIP(launch_zero(alpha, (size_t)sp.K * sp.m * 8, st));
    TNSLQ_HIP(launch_zero(beta, (size_t)sp.K * (sp.m + 1) * 8, st));
    TNSLQ_HIP(launch_zero(F, (size_t)sp.K * sp.m * 8, st));
    TNSLQ_HIP(launch_probe_init(TNSLQ_FP64, z, opt->seed, offset, 0, Q, nullptr, 0, alpha, beta, st));
    TNSLQ_HIP(hipEventRecord(e1, st));
    auto slot_of = [&](int jj) { return sp.reorth ? jj : jj % 3; };
    for (int j = 1; j <= sp.m; ++j) {
        double2 *q_cur = Q + slot_of(j - 1) * slot;
        double2 *q_prev = j > 1 ? Q + slot_of(j - 2) * slot : q_cur;
        double2 *q_next = Q + slot_of(j) * slot;
        TNSLQ_HIP(hipEventRecord(mv0[j], st));
        // Z = Psi^dagger q over P1 (d x d_R); Y = Psi Z over P2 = Psi^T (d_R x d)
        TNSLQ_HIP(launch_colmac(sp.dtype, 1, plain_colmac(P1, sp.d, sp.dR, q_cur, sp.K, Zp, sp.S1), st));
        TNSLQ_HIP(launch_sum_splits(Zp, sp.S1, (int64_t)sp.K * sp.dR, Z, st));
        TNSLQ_HIP(launch_colmac(sp.dtype, 0, plain_colmac(P2, sp.dR, sp.d, Z, sp.K, Yp, sp.S2), st));
        TNSLQ_HIP(hipEventRecord(mv1[j], st));
        TNSLQ_HIP(launch_passA(1, z, Yp, sp.S2, slot, 0, sp.K, q_prev, q_cur, w, alpha, beta, j, dotpart, st));
        TNSLQ_HIP(launch_passB(z, dotpart, q_cur, w, alpha, beta, j, nrmpart, sp.reorth ? 0 : 1, st));
        if (sp.reorth) TNSLQ_HIP(launch_reorth(z, Q, j, slot, w, hpart, h, alpha, beta, j, nrmpart, st));
        TNSLQ_HIP(launch_passC(TNSLQ_FP64, z, nrmpart, w, q_next, nullptr, 0, alpha, beta, j, st));
        TNSLQ_HIP(hipEventRecord(lz1[j], st));
    }
    TNSLQ_HIP(launch_steps(alpha, beta, sp.K, sp.m, sp.m, steps, st));
    TNSLQ_HIP(launch_quadrature(alpha, beta, steps, sp.K, sp.m, 1, sp.m, sp.fn, F, st));
    TNSLQ_HIP(launch_stats(beta, F, sp.K, sp.m, sp.m, G, stats, st));
    double sv[4];
    std::vector<int> hsteps(sp.K);
    TNSLQ_HIP(hipMemcpyAsync(sv, stats + (size_t)(sp.m - 1) * 4, sizeof sv, hipMemcpyDeviceToHost, st));
    TNSLQ_HIP(hipMemcpyAsync(hsteps.data(), steps, sizeof(int) * sp.K, hipMemcpyDeviceToHost, st));
    if (Gh) TNSLQ_HIP(hipMemcpyAsync(Gh, G, sizeof(double) * sp.K, hipMemcpyDeviceToHost, st));
    if (alh) TNSLQ_HIP(hipMemcpyAsync(alh, alpha, sizeof(double) * sp.K * sp.m, hipMemcpyDeviceToHost, st));
    if (beh) TNSLQ_HIP(hipMemcpyAsync(beh, beta, sizeof(double) * sp.K * (sp.m + 1), hipMemcpyDeviceToHost, st));
    if (Fh) TNSLQ_HIP(hipMemcpyAsync(Fh, F, sizeof(double) * sp.K * sp.m, hipMemcpyDeviceToHost, st));
    TNSLQ_HIP(hipStreamSynchronize(st));
    if (sth) std::copy(hsteps.begin(), hsteps.end(), sth);
    memset(res, 0, sizeof *res);
    res->value = sv[0];
    res->value_se = sv[1];
    res->steps_done = sp.m;
    res->steps_min = *std::min_element(hsteps.begin(), hsteps.end());
    res->complement = sp.complement;
    res->n_qubits_side = sp.n_side;
    res->t_layout_ms = elapsed(e0, e1);
    for (int j = 1; j <= sp.m; ++j) {
        res->t_matvec_ms += elapsed(mv0[j], mv1[j]);
        res->t_lanczos_ms += elapsed(mv1[j], lz1[j]);
    }
    res->t_total_ms = tm.ms();
    if (!std::isfinite(res->value)) return fail(TNSLQ_E_NONFINITE, "estimate is not finite");
    return TNSLQ_OK;
}

int spectral_sum(const void *psi, int dtype, int L, const int *s, int n_s, int fn, const tnslq_options *opt,
                 uint64_t offset, void *ws, size_t ws_bytes, void *stream, tnslq_spectral_result *res, double *Gh,
                 double *alh, double *beh, double *Fh, int *sth) {
    Timer tm;
    int rc;
    if (!res) return fail(TNSLQ_E_ARG, "result is NULL");
    if ((rc = check_dtype(dtype)) || (rc = check_subsystem(L, s, n_s)) || (rc = check_spectral_options(opt, fn)))
        return rc;
    if (n_s == 0 || n_s == L) {
        spectral_trivial(nullptr, fn, opt, res, Gh, alh, beh, Fh, sth);
        res->t_total_ms = tm.ms();
        return TNSLQ_OK;
    }
    SPlan sp;
    if ((rc = make_splan(dtype, L, s, n_s, opt, fn, sp))) return rc;
    if (!psi) return fail(TNSLQ_E_ARG, "psi is NULL");
    if (!ws) return fail(TNSLQ_E_ARG, "workspace is NULL");
    if ((uintptr_t)ws % ALIGN) return fail(TNSLQ_E_ARG, "workspace not 256-byte aligned");
    if (ws_bytes < sp.total) return fail(TNSLQ_E_WORKSPACE, "workspace %zu bytes, need %zu", ws_bytes, sp.total);
    return spectral_run(sp, psi, opt, offset, ws, (hipStream_t)stream, res, Gh, alh, beh, Fh, sth, tm);
}

int spectral_bytes(int dtype, int L, const int *s, int n_s, const tnslq_options *opt, int fn, size_t *bytes) {
    int rc;
    if ((rc = check_dtype(dtype)) || (rc = check_subsystem(L, s, n_s)) || (rc = check_spectral_options(opt, fn)))
        return rc;
    if (n_s == 0 || n_s == L) {
        *bytes = 0;
        return TNSLQ_OK;
    }
    SPlan sp;
    if ((rc = make_splan(dtype, L, s, n_s, opt, fn, sp))) return rc;
    *bytes = sp.total;
    return TNSLQ_OK;
}

// ------------------------------------------------ block matvec entry points
// Plan of tnslq_ptmatvec / tnslq_ptmatvec_static after the argument checks
// (no device work).
int ptmatvec_plan(int dtype, const tnslq_partition *part, int n_vectors, const void *X_dev, const void *Y_dev,
                  int precision, int chunk_vectors, Plan &pl) {
    int rc;
    if ((rc = check_dtype(dtype)) || (rc = check_partition(part)) || (rc = check_prec(precision))) return rc;
    if (part->n_a == 0 || part->n_b == 0) return fail(TNSLQ_E_PARTITION, "matvec needs non-empty A and B");
    if (chunk_vectors < 0) return fail(TNSLQ_E_ARG, "chunk_vectors must be >= 0");
    if ((rc = make_plan(dtype, part, n_vectors, 1, 0, precision, 0, TNSLQ_OPERATOR_LAZY, pl, chunk_vectors)))
        return rc;
    if (!X_dev || !Y_dev) return fail(TNSLQ_E_ARG, "NULL device pointer");
    if (X_dev == Y_dev) return fail(TNSLQ_E_ARG, "X and Y alias");
    return TNSLQ_OK;
}

// Both contractions of Eq. 4 for the planned block on workspace `ws`
// (regrouping psi, loading the vectors, every probe chunk).
int ptmatvec_run(Ctx &c, const void *psi_dev, const void *X_dev, void *Y_dev, void *ws, hipStream_t st) {
    if (!psi_dev) return fail(TNSLQ_E_ARG, "NULL device pointer");
    bind(c, ws, st);
    const Plan &pl = c.pl;
    int rc;
    if ((rc = do_layout(c, psi_dev))) return rc;
    if (pl.stream) {
        TNSLQ_HIP(launch_load_vectors_plain((const double2 *)X_dev, pl.dA, pl.dB, pl.K, pl.swapped, c.Xs, c.st));
        if ((rc = stream_contract(c, c.Xs, nullptr, nullptr))) return rc;
        TNSLQ_HIP(launch_reduce_partials(1, pl.fused ? c.Ypart : (const void *)c.Ym, pl.fused ? pl.S : 1,
                                         (int64_t)pl.K * pl.dAB, pl.dA, pl.dB, pl.K, pl.swapped, (double2 *)Y_dev,
                                         c.st));
        return TNSLQ_OK;
    }
    TNSLQ_HIP(launch_load_vectors(pl.prec, (const double2 *)X_dev, pl.dA, pl.dB, pl.K, pl.swapped, c.Xt, c.pl.nst1, c.st));
    for (int k0 = 0; k0 < pl.K; k0 += pl.kc) {
        const int kcur = std::min(pl.kc, pl.K - k0);
        if ((rc = contract_chunk(c, k0, kcur, nullptr, nullptr))) return rc;
        TNSLQ_HIP(launch_reduce_partials(pl.prec == TNSLQ_FP64, c.Ypart, pl.S, (int64_t)pl.kc * pl.dAB, pl.dA, pl.dB,
                                         kcur, pl.swapped, (double2 *)Y_dev + (size_t)k0 * pl.dAB, c.st));
    }
    return TNSLQ_OK;
}

// The fixed scratch of tnslq_ptmatvec_static: one copy per GPU, held from the
// library's load until the process ends.  Host code never passes the array
// itself to the device; it passes the device address hipGetSymbolAddress
// returns for the current GPU, looked up once per GPU and kept.
static __device__ __align__(256) unsigned char scratch[TNSLQ_STATIC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[MAX_DEVICES] = {};

int static_scratch(void **out) {
    int dev = -1;
    TNSLQ_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEVICES) return fail(TNSLQ_E_DEVICE, "device %d outside [0, %d)", dev, MAX_DEVICES);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return fail(TNSLQ_E_DEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        if (!ptr || (uintptr_t)ptr % ALIGN) return fail(TNSLQ_E_DEVICE, "static scratch address %p unusable", ptr);
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return TNSLQ_OK;
}

}  // namespace

extern "C" {

const char *tnslq_status_str(int s) {
    switch (s) {
        case TNSLQ_OK: return "ok";
        case TNSLQ_E_ARG: return "invalid argument";
        case TNSLQ_E_PARTITION: return "invalid partition";
        case TNSLQ_E_DTYPE: return "invalid dtype";
        case TNSLQ_E_WORKSPACE: return "workspace too small";
        case TNSLQ_E_DEVICE: return "device error";
        case TNSLQ_E_NONFINITE: return "non-finite value";
        case TNSLQ_E_STATE: return "state not normalised";
        default: return "unknown status";
    }
}

const char *tnslq_last_error(void) { return g_err.c_str(); }

int tnslq_version(void) { return 4; }

int tnslq_workspace_bytes(int dtype, const tnslq_partition *part, const tnslq_options *opt, size_t *bytes) {
    int rc;
    if (!bytes) return fail(TNSLQ_E_ARG, "bytes is NULL");
    if ((rc = check_options(opt))) return rc;
    if ((rc = check_dtype(dtype)) || (rc = check_partition(part))) return rc;
    if (part->n_a == 0 || part->n_b == 0) {
        *bytes = 0;
        return TNSLQ_OK;
    }
    Plan pl;
    if ((rc = make_plan(dtype, part, opt->n_probes, opt->n_steps, opt->reorth, opt->precision, 1,
                         opt->operator_form, pl, opt->chunk_probes)))
        return rc;
    *bytes = pl.total;
    return TNSLQ_OK;
}

namespace {
// Algorithm 1's outer loop over probes (Sec. III), in blocks of K probes on
// one regrouped psi: each block runs until its Lanczos error meets the
// target (lanczos_converged), its fitted G_n and errors beta_1^2 sigma_n join
// those of the earlier blocks, and blocks are added until the estimate over
// all of them meets the combined target (hutchinson_converged with the
// Lanczos part added in quadrature) or the next block would pass max_probes.
// The block's estimates come from the device; their mean and spread over the
// few hundred probes at most are summed here.
int run_probe_loop(Run &r, const tnslq_options *opt, tnslq_result *res, double *G_host, const Timer &tm) {
    Ctx &c = r.c;
    const Plan &pl = c.pl;
    const int K = pl.K;
    const double ln2 = std::log(2.0), b1sq = (double)pl.dAB;   // ||phi||^2 of a unit-modulus probe
    std::vector<double> Gall, Sall, g(K), sg(K);
    std::vector<int> hsteps(K);
    int steps_min = pl.m, jmax = 0, nmv = 0;
    double tmv = 0.0, tc1 = 0.0, tc2 = 0.0, tlz = 0.0;
    double T = 0.0, se = std::nan(""), epsl = 0.0, E = std::nan(""), de = INFINITY;
    int rc;
    for (int b = 0;; ++b) {
        if (b > 0) {
            // the next block: fresh probes on the same regrouped psi
            TNSLQ_HIP(launch_zero(c.alpha, (size_t)K * pl.m * 8, c.st));
            TNSLQ_HIP(launch_zero(c.beta, (size_t)K * (pl.m + 1) * 8, c.st));
            TNSLQ_HIP(launch_zero(c.F, (size_t)K * pl.m * 8, c.st));
            TNSLQ_HIP(launch_probe_init(pl.prec, c.z, opt->seed, opt->probe_offset + (uint64_t)b * K, pl.swapped,
                                        c.Q, pl.stream ? nullptr : c.Xt, pl.nst1, c.alpha, c.beta, c.st));
            r.jdone = 0;
        }
        if ((rc = run_steps(r, opt->n_steps, opt->stop_tol, true))) return rc;
        if ((rc = fit_step(r, r.jdone, c.G))) return rc;
        TNSLQ_HIP(hipMemcpyAsync(g.data(), c.G, sizeof(double) * K, hipMemcpyDeviceToHost, c.st));
        TNSLQ_HIP(hipMemcpyAsync(sg.data(), c.fsig, sizeof(double) * K, hipMemcpyDeviceToHost, c.st));
        TNSLQ_HIP(hipMemcpyAsync(hsteps.data(), c.steps, sizeof(int) * K, hipMemcpyDeviceToHost, c.st));
        TNSLQ_HIP(hipStreamSynchronize(c.st));
        for (int j = 1; j <= r.jdone; ++j) {
            const StepEvents &e = r.se[j];
            tmv += elapsed(e.mv0(), e.mv1());
            for (int ch = 0; ch < e.nchunk; ++ch) {
                tc1 += elapsed(ch == 0 ? e.mv0() : e.pa(ch - 1), e.c1(ch));
                tc2 += elapsed(e.c1(ch), e.c2(ch));
            }
            tlz += elapsed(e.mv1(), e.lz1());
        }
        nmv += r.jdone;
        jmax = std::max(jmax, r.jdone);
        for (int k = 0; k < K; ++k) {
            Gall.push_back(g[k]);
            Sall.push_back(b1sq * sg[k]);
            steps_min = std::min(steps_min, hsteps[k]);
        }
        const double N = (double)Gall.size();
        T = 0.0;
        epsl = 0.0;
        for (size_t i = 0; i < Gall.size(); ++i) {
            T += Gall[i];
            epsl += Sall[i];
        }
        T /= N;
        epsl /= N;
        if (Gall.size() > 1) {
            double v = 0.0;
            for (double x : Gall) v += (x - T) * (x - T);
            se = std::sqrt(v / (N - 1.0) / N);
            de = std::sqrt(se * se + epsl * epsl) / (T * ln2);
        }
        E = std::log2(T);
        if (std::isfinite(E) && std::isfinite(de) && de <= opt->stop_tol * std::max(std::fabs(E), 1.0)) break;
        if ((int64_t)(b + 2) * K > opt->max_probes) break;
    }
    zero_result(res);
    res->trace_norm = T;
    res->trace_norm_se = se;
    res->logneg = E;
    res->logneg_se = se / (T * ln2);
    res->lanczos_err = epsl / (T * ln2);
    res->steps_done = jmax;
    res->steps_min = steps_min;
    res->swapped_ab = pl.swapped;
    res->streamed = pl.stream ? (pl.fused ? 2 : 1) : 0;
    res->explicit_operator = pl.expl;
    res->mps_matvec = pl.mpsf ? (pl.mnet ? TNSLQ_MPS_MATVEC_NETWORK : TNSLQ_MPS_MATVEC_FACTORS) : 0;
    res->n_probes_used = (int)Gall.size();
    res->n_matvecs = nmv;
    res->n_contract_launches = c.n_launch;
    res->t_layout_ms = elapsed(r.e_start, r.e_layout);
    res->t_matvec_ms = tmv;
    res->t_contract1_ms = tc1;
    res->t_contract2_ms = tc2;
    res->t_lanczos_ms = tlz;
    if (G_host) std::copy(Gall.begin(), Gall.end(), G_host);
    res->t_total_ms = tm.ms();
    if (!std::isfinite(res->logneg))
        return fail(TNSLQ_E_NONFINITE, "estimate is not finite (trace norm %g)", res->trace_norm);
    return TNSLQ_OK;
}
}  // namespace

int tnslq_logneg(const void *psi_dev, int dtype, const tnslq_partition *part, const tnslq_options *opt, void *ws_dev,
                 size_t ws_bytes, void *stream, tnslq_result *res, double *G_host, double *alpha_host,
                 double *beta_host, double *F_host, int *steps_host) {
    Timer tm;
    int rc;
    g_err.clear();
    if (!res) return fail(TNSLQ_E_ARG, "result is NULL");
    if ((rc = check_options(opt))) return rc;
    if ((rc = check_dtype(dtype)) || (rc = check_partition(part))) return rc;
    if (part->n_a == 0 || part->n_b == 0) return trivial(opt, res, G_host, alpha_host, beta_host, F_host, steps_host);
    const bool loop = opt->max_probes > opt->n_probes;
    if (loop && (alpha_host || beta_host || F_host || steps_host))
        return fail(TNSLQ_E_ARG, "with max_probes > n_probes only G_host may be requested");
    Run r;
    if ((rc = run_begin(r, dtype, part, opt, psi_dev, ws_dev, ws_bytes, stream))) return rc;
    if (loop) return run_probe_loop(r, opt, res, G_host, tm);
    if ((rc = run_steps(r, opt->n_steps, opt->stop_tol))) return rc;
    return run_finish(r, res, G_host, alpha_host, beta_host, F_host, steps_host, tm);
}

int tnslq_workspace_bytes_dims(int dtype, const tnslq_partition_dims *part, const tnslq_options *opt,
                               size_t *bytes) {
    int rc;
    if (!bytes) return fail(TNSLQ_E_ARG, "bytes is NULL");
    if ((rc = check_options(opt)) || (rc = check_dtype(dtype)) || (rc = check_partition_dims(part))) return rc;
    if (part->n_a == 0 || part->n_b == 0) {
        *bytes = 0;
        return TNSLQ_OK;
    }
    Plan pl;
    if ((rc = make_plan_dims(dtype, part, opt->n_probes, opt->n_steps, opt->reorth, opt->precision, 1,
                             opt->operator_form, pl)))
        return rc;
    *bytes = pl.total;
    return TNSLQ_OK;
}

int tnslq_logneg_dims(const void *psi_dev, int dtype, const tnslq_partition_dims *part, const tnslq_options *opt,
                      void *ws_dev, size_t ws_bytes, void *stream, tnslq_result *res, double *G_host,
                      double *alpha_host, double *beta_host, double *F_host, int *steps_host) {
    Timer tm;
    int rc;
    g_err.clear();
    if (!res) return fail(TNSLQ_E_ARG, "result is NULL");
    if ((rc = check_options(opt)) || (rc = check_dtype(dtype)) || (rc = check_partition_dims(part))) return rc;
    if (part->n_a == 0 || part->n_b == 0) return trivial(opt, res, G_host, alpha_host, beta_host, F_host, steps_host);
    const bool loop = opt->max_probes > opt->n_probes;
    if (loop && (alpha_host || beta_host || F_host || steps_host))
        return fail(TNSLQ_E_ARG, "with max_probes > n_probes only G_host may be requested");
    Run r;
    if ((rc = make_plan_dims(dtype, part, opt->n_probes, opt->n_steps, opt->reorth, opt->precision, 1,
                             opt->operator_form, r.c.pl)))
        return rc;
    if ((rc = run_start(r, opt, psi_dev, ws_dev, ws_bytes, stream))) return rc;
    if (loop) return run_probe_loop(r, opt, res, G_host, tm);
    if ((rc = run_steps(r, opt->n_steps, opt->stop_tol))) return rc;
    return run_finish(r, res, G_host, alpha_host, beta_host, F_host, steps_host, tm);
}

int tnslq_ptmatvec_workspace_bytes(int dtype, const tnslq_partition *part, int n_vectors, int precision,
                                   int chunk_vectors, size_t *bytes) {
    int rc;
    if (!bytes) return fail(TNSLQ_E_ARG, "bytes is NULL");
    if ((rc = check_dtype(dtype)) || (rc = check_partition(part)) || (rc = check_prec(precision))) return rc;
    if (part->n_a == 0 || part->n_b == 0) return fail(TNSLQ_E_PARTITION, "matvec needs non-empty A and B");
    Plan pl;
    if (chunk_vectors < 0) return fail(TNSLQ_E_ARG, "chunk_vectors must be >= 0");
    if ((rc = make_plan(dtype, part, n_vectors, 1, 0, precision, 0, TNSLQ_OPERATOR_LAZY, pl, chunk_vectors))) return rc;
    *bytes = pl.total;
    return TNSLQ_OK;
}

int tnslq_ptmatvec(const void *psi_dev, int dtype, const tnslq_partition *part, int n_vectors, const void *X_dev,
                   void *Y_dev, int precision, int chunk_vectors, void *ws_dev, size_t ws_bytes, void *stream) {
    g_err.clear();
    Ctx c;
    int rc;
    if ((rc = ptmatvec_plan(dtype, part, n_vectors, X_dev, Y_dev, precision, chunk_vectors, c.pl))) return rc;
    if (!ws_dev) return fail(TNSLQ_E_ARG, "NULL device pointer");
    if ((uintptr_t)ws_dev % ALIGN) return fail(TNSLQ_E_ARG, "workspace not 256-byte aligned");
    if (ws_bytes < c.pl.total) return fail(TNSLQ_E_WORKSPACE, "workspace %zu bytes, need %zu", ws_bytes, c.pl.total);
    return ptmatvec_run(c, psi_dev, X_dev, Y_dev, ws_dev, (hipStream_t)stream);
}

int tnslq_ptmatvec_static(const void *psi_dev, int dtype, const tnslq_partition *part, int n_vectors,
                          const void *X_dev, void *Y_dev, int precision, int chunk_vectors, void *stream) {
    g_err.clear();
    Ctx c;
    int rc;
    if ((rc = ptmatvec_plan(dtype, part, n_vectors, X_dev, Y_dev, precision, chunk_vectors, c.pl))) return rc;
    if (c.pl.total > TNSLQ_STATIC_SCRATCH_BYTES)
        return fail(TNSLQ_E_WORKSPACE, "problem needs %zu bytes of scratch, the static scratch holds %zu", c.pl.total,
                    (size_t)TNSLQ_STATIC_SCRATCH_BYTES);
    void *ws = nullptr;
    if ((rc = static_scratch(&ws))) return rc;
    return ptmatvec_run(c, psi_dev, X_dev, Y_dev, ws, (hipStream_t)stream);
}

int tnslq_spectral_workspace_bytes(int dtype, int n_qubits, const int *s, int n_s, const tnslq_options *opt,
                                   size_t *bytes) {
    g_err.clear();
    if (!bytes) return fail(TNSLQ_E_ARG, "bytes is NULL");
    // the function does not change the workspace; entropy stands for both
    return spectral_bytes(dtype, n_qubits, s, n_s, opt, TNSLQ_F_ENTROPY, bytes);
}

int tnslq_spectral_sum(const void *psi_dev, int dtype, int n_qubits, const int *s, int n_s, int fn,
                       const tnslq_options *opt, void *ws_dev, size_t ws_bytes, void *stream,
                       tnslq_spectral_result *res, double *G_host, double *alpha_host, double *beta_host,
                       double *F_host, int *steps_host) {
    g_err.clear();
    if (!opt) return fail(TNSLQ_E_ARG, "options is NULL");
    return spectral_sum(psi_dev, dtype, n_qubits, s, n_s, fn, opt, opt->probe_offset, ws_dev, ws_bytes, stream, res,
                        G_host, alpha_host, beta_host, F_host, steps_host);
}

int tnslq_mutual_information_workspace_bytes(int dtype, const tnslq_partition *part, const tnslq_options *opt,
                                             size_t *bytes) {
    int rc;
    g_err.clear();
    if (!bytes) return fail(TNSLQ_E_ARG, "bytes is NULL");
    if ((rc = check_partition(part))) return rc;
    std::vector<int> ab(part->a, part->a + part->n_a);
    ab.insert(ab.end(), part->b, part->b + part->n_b);
    size_t best = 0, b = 0;
    const int *sets[3] = {part->a, part->b, ab.data()};
    const int sizes[3] = {part->n_a, part->n_b, (int)ab.size()};
    for (int i = 0; i < 3; ++i) {
        if ((rc = spectral_bytes(dtype, part->n_qubits, sets[i], sizes[i], opt, TNSLQ_F_ENTROPY, &b))) return rc;
        best = std::max(best, b);
    }
    *bytes = best;
    return TNSLQ_OK;
}

int tnslq_mutual_information(const void *psi_dev, int dtype, const tnslq_partition *part, const tnslq_options *opt,
                             void *ws_dev, size_t ws_bytes, void *stream, double *out) {
    int rc;
    g_err.clear();
    if (!out) return fail(TNSLQ_E_ARG, "out is NULL");
    if (!opt) return fail(TNSLQ_E_ARG, "options is NULL");
    if ((rc = check_partition(part))) return rc;
    std::vector<int> ab(part->a, part->a + part->n_a);
    ab.insert(ab.end(), part->b, part->b + part->n_b);
    const int *sets[3] = {part->a, part->b, ab.data()};
    const int sizes[3] = {part->n_a, part->n_b, (int)ab.size()};
    double v[3], e[3];
    for (int i = 0; i < 3; ++i) {
        tnslq_spectral_result r;
        const uint64_t off = opt->probe_offset + (uint64_t)i * (uint64_t)opt->n_probes;
        if ((rc = spectral_sum(psi_dev, dtype, part->n_qubits, sets[i], sizes[i], TNSLQ_F_ENTROPY, opt, off, ws_dev,
                               ws_bytes, stream, &r, nullptr, nullptr, nullptr, nullptr, nullptr)))
            return rc;
        v[i] = r.value;
        e[i] = (sizes[i] == 0 || sizes[i] == part->n_qubits) ? 0.0 : r.value_se;
    }
    out[0] = v[0] + v[1] - v[2];
    out[1] = std::sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
    for (int i = 0; i < 3; ++i) {
        out[2 + 2 * i] = v[i];
        out[3 + 2 * i] = e[i];
    }
    return TNSLQ_OK;
}

namespace {
// Roles, sizes and workspace of tnslq_rho_pt: P and its conjugate as FP64
// bricks, then the dense FP64 product.
struct PtPlan {
    Plan pl;
    size_t off_Pabe = 0, off_Pabc = 0, off_Cd = 0, total = 0;
};
int pt_offsets(PtPlan &pp) {
    const Plan &pl = pp.pl;
    const size_t pb = up(brick_bytes(TNSLQ_FP64, pl.dAB, pl.dE));
    pp.off_Pabe = 0;
    pp.off_Pabc = pb;
    pp.off_Cd = 2 * pb;
    pp.total = pp.off_Cd + up((size_t)(pl.dAB * pl.dAB) * 16);
    return TNSLQ_OK;
}
int make_pt_plan(int dtype, const tnslq_partition *part, PtPlan &pp) {
    int rc;
    if ((rc = check_dtype(dtype)) || (rc = check_partition(part))) return rc;
    if (part->n_a == 0 || part->n_b == 0) return fail(TNSLQ_E_PARTITION, "rho_pt needs non-empty A and B");
    if (part->n_a + part->n_b > 14)
        return fail(TNSLQ_E_ARG, "rho_pt: d_A d_B = 2^%d exceeds %lld", part->n_a + part->n_b,
                    (long long)EXPLICIT_MAX_N);
    if ((rc = make_plan(dtype, part, 1, 1, 0, TNSLQ_FP64, 1, TNSLQ_OPERATOR_EXPLICIT, pp.pl))) return rc;
    return pt_offsets(pp);
}
int make_pt_plan_dims(int dtype, const tnslq_partition_dims *part, PtPlan &pp) {
    int rc;
    if ((rc = check_dtype(dtype)) || (rc = check_partition_dims(part))) return rc;
    if (part->n_a == 0 || part->n_b == 0) return fail(TNSLQ_E_PARTITION, "rho_pt needs non-empty A and B");
    if ((rc = make_plan_dims(dtype, part, 1, 1, 0, TNSLQ_FP64, 1, TNSLQ_OPERATOR_EXPLICIT, pp.pl))) return rc;
    return pt_offsets(pp);
}
int rho_pt_run(const PtPlan &pp, const void *psi_dev, void *rho_dev, void *ws_dev, size_t ws_bytes, void *stream) {
    int rc;
    if (!psi_dev || !rho_dev || !ws_dev) return fail(TNSLQ_E_ARG, "NULL device pointer");
    if ((uintptr_t)ws_dev % ALIGN) return fail(TNSLQ_E_ARG, "workspace not 256-byte aligned");
    if (ws_bytes < pp.total) return fail(TNSLQ_E_WORKSPACE, "workspace %zu bytes, need %zu", ws_bytes, pp.total);
    const Plan &pl = pp.pl;
    char *ws = (char *)ws_dev;
    hipStream_t st = (hipStream_t)stream;
    if ((rc = form_rho(pl, TNSLQ_FP64, psi_dev, ws + pp.off_Pabe, ws + pp.off_Pabc, ws + pp.off_Cd, st))) return rc;
    TNSLQ_HIP(launch_pt_dense((const double2 *)(ws + pp.off_Cd), pl.dAB, pl.dB, (double2 *)rho_dev, st));
    return TNSLQ_OK;
}
}  // namespace

int tnslq_rho_pt_workspace_bytes(int dtype, const tnslq_partition *part, size_t *bytes) {
    int rc;
    if (!bytes) return fail(TNSLQ_E_ARG, "bytes is NULL");
    PtPlan pp;
    if ((rc = make_pt_plan(dtype, part, pp))) return rc;
    *bytes = pp.total;
    return TNSLQ_OK;
}

int tnslq_rho_pt(const void *psi_dev, int dtype, const tnslq_partition *part, void *rho_dev, void *ws_dev,
                 size_t ws_bytes, void *stream) {
    int rc;
    g_err.clear();
    PtPlan pp;
    if ((rc = make_pt_plan(dtype, part, pp))) return rc;
    return rho_pt_run(pp, psi_dev, rho_dev, ws_dev, ws_bytes, stream);
}

int tnslq_rho_pt_dims_workspace_bytes(int dtype, const tnslq_partition_dims *part, size_t *bytes) {
    int rc;
    if (!bytes) return fail(TNSLQ_E_ARG, "bytes is NULL");
    PtPlan pp;
    if ((rc = make_pt_plan_dims(dtype, part, pp))) return rc;
    *bytes = pp.total;
    return TNSLQ_OK;
}

int tnslq_rho_pt_dims(const void *psi_dev, int dtype, const tnslq_partition_dims *part, void *rho_dev, void *ws_dev,
                      size_t ws_bytes, void *stream) {
    int rc;
    g_err.clear();
    PtPlan pp;
    if ((rc = make_pt_plan_dims(dtype, part, pp))) return rc;
    return rho_pt_run(pp, psi_dev, rho_dev, ws_dev, ws_bytes, stream);
}

// ------------------------------------------------------------ MPS blocks
int tnslq_mps_effective_state_size(const tnslq_mps *mps, int a0, int n_a, int b0, int n_b, int *q, size_t *ws_bytes) {
    int rc;
    g_err.clear();
    if (!q || !ws_bytes) return fail(TNSLQ_E_ARG, "NULL output");
    MpsPlan mp;
    if ((rc = plan_mps(mps, a0, n_a, b0, n_b, mp))) return rc;
    for (int i = 0; i < 3; ++i) q[i] = mp.q[i];
    *ws_bytes = mp.total;
    return TNSLQ_OK;
}

int tnslq_mps_effective_state(const tnslq_mps *mps, int a0, int n_a, int b0, int n_b, void *psi_dev, void *ws_dev,
                              size_t ws_bytes, void *stream) {
    int rc;
    g_err.clear();
    MpsPlan mp;
    if ((rc = plan_mps(mps, a0, n_a, b0, n_b, mp))) return rc;
    if (!mps->tensors || !psi_dev || !ws_dev) return fail(TNSLQ_E_ARG, "NULL device pointer");
    if ((uintptr_t)ws_dev % ALIGN) return fail(TNSLQ_E_ARG, "workspace not 256-byte aligned");
    if (ws_bytes < mp.total) return fail(TNSLQ_E_WORKSPACE, "workspace %zu bytes, need %zu", ws_bytes, mp.total);
    hipStream_t st = (hipStream_t)stream;
    char *ws = (char *)ws_dev;
    MpsFactors f;
    if ((rc = mps_build(mp, (const double2 *)mps->tensors, ws, st, f))) return rc;
    // psi[(kA, u')][(kB, v)] = sum_m P[(kA, u')][m] Qp[m][(kB, v)]
    const int64_t nrow = f.kA * f.Up, ncol = f.kB * f.V;
    double2 *Tout = (double2 *)(ws + mp.off_T);
    TNSLQ_HIP(launch_zgemm(0, 0, f.P, f.Qp, Tout, (int)nrow, (int)ncol, (int)f.M, f.M, ncol, ncol, 1, 0, 0, 0, st));
    double *part = (double *)(ws + mp.off_part);
    TNSLQ_HIP(launch_sumsq(Tout, nrow * ncol, part, st));
    TNSLQ_HIP(launch_assemble(Tout, mp.kA, 1, mp.Up, mp.kB, mp.Vf, int64_t(1) << mp.q[0], int64_t(1) << mp.q[1],
                              int64_t(1) << mp.q[2], part + 256, (double2 *)psi_dev, st));
    return mps_check(mp, ws, st);
}

// Plan of Algorithm 1 on the two-block operator in factorised form: the
// Lanczos vectors run over (a, b) of the blocks' compressed physical indices.
static int make_plan_mpsf(const tnslq_mps *mps, int a0, int n_a, int b0, int n_b, const tnslq_options *opt, MpsPlan &mp,
                   Plan &pl) {
    int rc;
    if ((rc = check_options(opt))) return rc;
    if (opt->precision != TNSLQ_FP64 && opt->precision != TNSLQ_FP32)
        return fail(TNSLQ_E_ARG, "the factorised MPS operator computes in FP64 or FP32 (precision %d)",
                    opt->precision);
    if (opt->operator_form != TNSLQ_OPERATOR_AUTO)
        return fail(TNSLQ_E_ARG, "operator_form must be TNSLQ_OPERATOR_AUTO for MPS blocks");
    if (!mps) return fail(TNSLQ_E_ARG, "mps is NULL");
    if (mps->matvec < TNSLQ_MPS_MATVEC_AUTO || mps->matvec > TNSLQ_MPS_MATVEC_NETWORK)
        return fail(TNSLQ_E_ARG, "matvec %d is not a TNSLQ_MPS_MATVEC_ value", mps->matvec);
    if ((rc = plan_mps(mps, a0, n_a, b0, n_b, mp, false, true))) return rc;
    // complex multiply-adds per probe and matvec of the two forms
    const bool gap = mp.b0 > mp.a1;
    const double kA = (double)mp.kA, kB = (double)mp.kB;
    const double UpM = (double)mp.Up * mp.Mf, MV = (double)mp.Mf * mp.Vf;
    const double UM = (double)mp.U * mp.Mb, NV = (double)mp.Nb * mp.V, MN = (double)mp.Mb * mp.Nb,
                 UV = (double)mp.U * mp.V;
    const double c_pq = UpM * kB * kA + UpM * MV * kB + kA * MV * UpM + kA * kB * MV;
    const double c_net = UM * kB * kA + UM * NV * kB + (gap ? MN * MN * UV : 0.0) + (mp.closed ? UV * UV * MN : 0.0) +
                         kA * NV * UM + kA * kB * NV;
    // the network's layout scratch: four tensors of (bond^2)^2 entries
    const double wmax = std::max({UM, NV, MN, UV, (double)mp.U * mp.Nb});
    const bool net_fits = 4.0 * wmax * wmax * 16.0 <= (double)(size_t(64) << 30);
    if (mps->matvec == TNSLQ_MPS_MATVEC_NETWORK && !net_fits)
        return fail(TNSLQ_E_ARG, "the network form's layout would need more than 64 GiB");
    bool net = mps->matvec == TNSLQ_MPS_MATVEC_NETWORK ||
               (mps->matvec == TNSLQ_MPS_MATVEC_AUTO && net_fits && c_net < c_pq);
    if (!net) {
        MpsPlan mq;
        if ((rc = plan_mps(mps, a0, n_a, b0, n_b, mq, false, false))) {
            if (mps->matvec == TNSLQ_MPS_MATVEC_FACTORS || !net_fits) return rc;
            net = true;   // the factors would not fit the products' index range
            g_err.clear();
        } else {
            mp = mq;
        }
    }
    pl = Plan();
    pl.mpsf = 1;
    pl.mnet = net;
    pl.ngap = gap;
    pl.nring = mp.closed;
    pl.nU = mp.U;
    pl.nM = mp.Mb;
    pl.nN = mp.Nb;
    pl.nV = mp.V;
    pl.dtype = TNSLQ_C128;
    pl.prec = opt->precision;
    pl.K = opt->n_probes;
    pl.m = opt->n_steps;
    pl.reorth = opt->reorth;
    pl.dA = mp.kA;
    pl.dB = mp.kB;
    pl.dAB = mp.kA * mp.kB;
    pl.mUp = mp.Up;
    pl.mM = mp.Mf;
    pl.mV = mp.Vf;
    pl.dE = mp.Up * mp.Vf;
    pl.D = pl.dAB * pl.dE;
    pl.mps_bytes = mp.total;
    return plan_rest(pl, TNSLQ_C128, pl.prec, pl.K, 1);
}

int tnslq_workspace_bytes_mps(const tnslq_mps *mps, int a0, int n_a, int b0, int n_b, const tnslq_options *opt,
                              size_t *bytes) {
    int rc;
    g_err.clear();
    if (!bytes) return fail(TNSLQ_E_ARG, "bytes is NULL");
    MpsPlan mp;
    Plan pl;
    if ((rc = make_plan_mpsf(mps, a0, n_a, b0, n_b, opt, mp, pl))) return rc;
    *bytes = pl.total;
    return TNSLQ_OK;
}

int tnslq_logneg_mps(const tnslq_mps *mps, int a0, int n_a, int b0, int n_b, const tnslq_options *opt, void *ws_dev,
                     size_t ws_bytes, void *stream, tnslq_result *res, double *G_host, double *alpha_host,
                     double *beta_host, double *F_host, int *steps_host) {
    Timer tm;
    int rc;
    g_err.clear();
    if (!res) return fail(TNSLQ_E_ARG, "result is NULL");
    MpsPlan mp;
    Run r;
    if ((rc = make_plan_mpsf(mps, a0, n_a, b0, n_b, opt, mp, r.c.pl))) return rc;
    if (!mps->tensors) return fail(TNSLQ_E_ARG, "tensors is NULL");
    const bool loop = opt->max_probes > opt->n_probes;
    if (loop && (alpha_host || beta_host || F_host || steps_host))
        return fail(TNSLQ_E_ARG, "with max_probes > n_probes only G_host may be requested");
    r.c.mp = &mp;
    if ((rc = run_start(r, opt, mps->tensors, ws_dev, ws_bytes, stream))) return rc;
    if (loop) return run_probe_loop(r, opt, res, G_host, tm);
    if ((rc = run_steps(r, opt->n_steps, opt->stop_tol))) return rc;
    return run_finish(r, res, G_host, alpha_host, beta_host, F_host, steps_host, tm);
}

int tnslq_quadrature(const double *alpha_dev, const double *beta_dev, const int *steps_dev, int n_probes, int n_steps,
                     double *F_dev, void *stream) {
    g_err.clear();
    if (!alpha_dev || !beta_dev || !F_dev) return fail(TNSLQ_E_ARG, "NULL device pointer");
    if (n_probes < 1 || n_steps < 1 || n_steps > TNSLQ_MAX_STEPS) return fail(TNSLQ_E_ARG, "bad sizes");
    TNSLQ_HIP(launch_quadrature(alpha_dev, beta_dev, steps_dev, n_probes, n_steps, 1, n_steps, TNSLQ_F_ABS, F_dev,
                                (hipStream_t)stream));
    return TNSLQ_OK;
}

int tnslq_probes(uint64_t seed, uint64_t probe_offset, int n_probes, int64_t d, void *X_dev, void *stream) {
    g_err.clear();
    if (!X_dev) return fail(TNSLQ_E_ARG, "X is NULL");
    if (n_probes < 1 || n_probes > 65535 || d < 1) return fail(TNSLQ_E_ARG, "bad sizes");
    TNSLQ_HIP(launch_probes_plain(seed, probe_offset, n_probes, d, (double2 *)X_dev, (hipStream_t)stream));
    return TNSLQ_OK;
}

int tnslq_mlp_workspace_bytes(int batch, size_t *bytes) {
    if (!bytes) return fail(TNSLQ_E_ARG, "bytes is NULL");
    if (batch < 1) return fail(TNSLQ_E_ARG, "batch must be >= 1");
    *bytes = mlp_ws_bytes(batch);
    return TNSLQ_OK;
}

int tnslq_mlp_forward(const float *params, const float *norm, const float *x, int batch, float *out, void *ws,
                      size_t ws_bytes, void *stream) {
    g_err.clear();
    if (!params || !norm || !x || !out || !ws) return fail(TNSLQ_E_ARG, "NULL device pointer");
    if (batch < 1 || batch > (1 << 20)) return fail(TNSLQ_E_ARG, "batch %d outside [1, 2^20]", batch);
    if (ws_bytes < mlp_ws_bytes(batch)) return fail(TNSLQ_E_WORKSPACE, "workspace too small");
    TNSLQ_HIP(mlp_forward(params, norm, x, batch, out, ws, (hipStream_t)stream));
    return TNSLQ_OK;
}

int tnslq_mlp_loss_grad(const float *params, const float *norm, const float *x, const float *r, int batch,
                        float *loss, float *grad, void *ws, size_t ws_bytes, void *stream) {
    g_err.clear();
    if (!params || !norm || !x || !r || !grad || !ws) return fail(TNSLQ_E_ARG, "NULL device pointer");
    if (batch < 1 || batch > (1 << 20)) return fail(TNSLQ_E_ARG, "batch %d outside [1, 2^20]", batch);
    if (ws_bytes < mlp_ws_bytes(batch)) return fail(TNSLQ_E_WORKSPACE, "workspace too small");
    TNSLQ_HIP(mlp_loss_grad(params, norm, x, r, nullptr, batch, loss, grad, ws, (hipStream_t)stream));
    return TNSLQ_OK;
}

int tnslq_mlp_adam(float *params, float *m, float *v, const float *grad, int t, float lr, void *stream) {
    g_err.clear();
    if (!params || !m || !v || !grad) return fail(TNSLQ_E_ARG, "NULL device pointer");
    if (t < 1) return fail(TNSLQ_E_ARG, "t must be >= 1");
    TNSLQ_HIP(mlp_adam(params, m, v, grad, TNSLQ_MLP_NPARAMS, t, lr, (hipStream_t)stream));
    return TNSLQ_OK;
}

int tnslq_mlp_train(float *params, float *m, float *v, const float *norm, const float *x, const float *r,
                    const int *idx, int batch, int n_batches, int t0, float lr, float *losses, void *ws,
                    size_t ws_bytes, void *stream) {
    g_err.clear();
    if (!params || !m || !v || !norm || !x || !r || !idx || !ws) return fail(TNSLQ_E_ARG, "NULL device pointer");
    if (batch < 1 || batch > (1 << 20) || n_batches < 0 || t0 < 1) return fail(TNSLQ_E_ARG, "bad sizes");
    const size_t need = mlp_ws_bytes(batch) + (size_t)TNSLQ_MLP_NPARAMS * 4 + 256;
    if (ws_bytes < need) return fail(TNSLQ_E_WORKSPACE, "workspace %zu bytes, need %zu", ws_bytes, need);
    hipStream_t st = (hipStream_t)stream;
    float *grad = (float *)((char *)ws + (mlp_ws_bytes(batch) + 255) / 256 * 256);
    for (int s = 0; s < n_batches; ++s) {
        TNSLQ_HIP(mlp_loss_grad(params, norm, x, r, idx + (size_t)s * batch, batch, losses ? losses + s : nullptr,
                                grad, ws, st));
        TNSLQ_HIP(mlp_adam(params, m, v, grad, TNSLQ_MLP_NPARAMS, t0 + s, lr, st));
    }
    return TNSLQ_OK;
}

int tnslq_logneg_surrogate(const void *psi_dev, int dtype, const tnslq_partition *part, const tnslq_options *opt,
                           const float *params, const float *norm, float y_scale, int early_steps, double tol,
                           void *ws_dev, size_t ws_bytes, void *stream, tnslq_result *res, double *info) {
    Timer tm;
    int rc;
    g_err.clear();
    if (!res || !info || !params || !norm) return fail(TNSLQ_E_ARG, "NULL pointer");
    if ((rc = check_options(opt))) return rc;
    if (early_steps < TNSLQ_SURROGATE_MIN_EARLY || early_steps > TNSLQ_SURROGATE_MAX_EARLY)
        return fail(TNSLQ_E_ARG, "early_steps %d outside [%d, %d]", early_steps, TNSLQ_SURROGATE_MIN_EARLY,
                    TNSLQ_SURROGATE_MAX_EARLY);
    if (opt->max_probes > opt->n_probes) return fail(TNSLQ_E_ARG, "the surrogate runs one block of probes");
    if (opt->n_steps < early_steps) return fail(TNSLQ_E_ARG, "n_steps must be >= early_steps");
    if (!(tol > 0.0)) return fail(TNSLQ_E_ARG, "tol must be > 0");
    if ((rc = check_dtype(dtype)) || (rc = check_partition(part))) return rc;
    if (part->n_a == 0 || part->n_b == 0) {
        info[0] = 0.0;
        info[1] = 0.0;
        info[2] = 0.0;
        info[3] = 0.0;
        info[4] = 0.0;
        return trivial(opt, res, nullptr, nullptr, nullptr, nullptr, nullptr);
    }
    Run r;
    if ((rc = run_begin(r, dtype, part, opt, psi_dev, ws_dev, ws_bytes, stream))) return rc;
    if ((rc = run_steps(r, early_steps, 0.0))) return rc;
    Ctx &c = r.c;
    const Plan &pl = c.pl;
    if ((rc = quad_stats(c, r.jdone, r.jdone, r.jdone, r.jdone, nullptr))) return rc;
    // features in the caller's roles (log2 d_A, log2 d_B as given)
    const double dA = double(int64_t(1) << part->n_a), dB = double(int64_t(1) << part->n_b);
    TNSLQ_HIP(launch_features(c.alpha, c.beta, pl.K, pl.m, early_steps, double(pl.dAB), dA, dB, double(pl.dE), c.feat,
                              c.st));
    float *out = c.feat + 32;
    TNSLQ_HIP(mlp_forward(params, norm, c.feat, 1, out, c.mlpws, c.st));
    float u[2];
    double s[4];
    TNSLQ_HIP(hipMemcpyAsync(u, out, sizeof u, hipMemcpyDeviceToHost, c.st));
    TNSLQ_HIP(hipMemcpyAsync(s, c.stats + (size_t)(r.jdone - 1) * 4, sizeof s, hipMemcpyDeviceToHost, c.st));
    TNSLQ_HIP(hipStreamSynchronize(c.st));
    const double e_early = s[2];
    const double mu = e_early + (double)y_scale * u[0];
    const double sigma = (double)y_scale * std::exp(0.5 * (double)u[1]);
    info[0] = mu;
    info[1] = sigma;
    info[2] = e_early;
    if (std::isfinite(mu) && std::isfinite(sigma) && sigma <= tol * std::max(std::fabs(mu), 1.0)) {
        if ((rc = run_finish(r, res, nullptr, nullptr, nullptr, nullptr, nullptr, tm))) return rc;
        res->logneg = mu;
        res->logneg_se = sigma;
        info[3] = 0.0;
        info[4] = std::nan("");
        return TNSLQ_OK;
    }
    if ((rc = run_steps(r, opt->n_steps, opt->stop_tol))) return rc;
    if ((rc = run_finish(r, res, nullptr, nullptr, nullptr, nullptr, nullptr, tm))) return rc;
    info[3] = 1.0;
    info[4] = res->logneg;
    return TNSLQ_OK;
}

}  // extern "C"
