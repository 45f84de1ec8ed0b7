// Internal declarations shared by the libtnslq translation units.
//
// Data layout in HBM.  The four operands of the two contractions are complex
// matrices of R rows by Kr reduction terms, stored in bricks (operands.h):
//   P_aeb   psi regrouped as (A, E, B): d_A rows a, reduction index (c, b')
//           (b' fastest) of the second contraction.
//   P_bea   psi regrouped as (B, E, A) and conjugated: d_B d_E rows (b, c),
//           reduction index a' of the first contraction.
//   Xt      the current Lanczos vectors: rows (k, b'), reduction index a'.
//   Ups     intermediary (i) of Sec. V: rows (k, b), reduction index (c, b'),
//           the B operand of the second contraction.
//   Ypart   FP32 or FP64 split-K partial sums of Y[k][a][b], interleaved
//           complex, row-major.
// Both contractions are therefore "NT" products C = A * B^T whose operands are
// bricked along the reduction index.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "operands.h"
#include "tnslq.h"

namespace tnslq {

// ------------------------------------------------------------ plan
// Sites of any local dimension (flat index of psi in mixed radix, site 0 most
// significant): groups A, B, E, each listing its sites' dimensions and psi
// index strides, most significant first.
struct MixedDesc {
    int n[3];
    int64_t d[3];
    int dim[3][TNSLQ_MAX_QUBITS];
    int64_t stride[3][TNSLQ_MAX_QUBITS];
};

struct Plan {
    int L = 0;
    int nA = 0, nB = 0, nE = 0;      // sizes in the roles used on the device
    int qa[TNSLQ_MAX_QUBITS], qb[TNSLQ_MAX_QUBITS], qe[TNSLQ_MAX_QUBITS];
    int swapped = 0;                 // roles of A and B exchanged
    int64_t dA = 1, dB = 1, dE = 1, dAB = 1, D = 1;
    int dtype = TNSLQ_C64;
    int prec = TNSLQ_FP32;
    int K = 1, m = 1, reorth = 0;
    int kc = 1;                      // probes per contraction chunk
    int kc_cap = 0;                  // caller's cap on kc (0: from the budget alone)
    int S = 1;                       // split-K factor of the second contraction
    int S1 = 1;                      // split-K factor of the first contraction
    int stream = 0;                  // contractions as two streaming passes over psi (K d_B <= 8)
    int S1s = 1, S2s = 1;            // row splits of the two streaming passes
    int fused = 0;                   // streaming regime in one read of psi (fused.hip)
    int two_pass = 0;                // caller asked for the two-pass streaming form
    int expl = 0;                    // rho^{T_B} formed explicitly (intermediary (iii))
    int64_t nst_rho = 1;             // bricks along the reduction index of the explicit matvec
    int64_t nst_e = 1;               // bricks along E of the forming product
    int mpsf = 0;                    // two-block MPS operator in factorised form (Sec. VI)
    int64_t mUp = 1, mM = 1, mV = 1; // its factors P[a][u'][m], Q[b][m][v]
    int mnet = 0;                    // ... applied as the network R_A, E_W, E_Z, R_B instead
    int ngap = 0, nring = 0;         // the network's traced gap and ring sections
    int64_t nU = 1, nM = 1, nN = 1, nV = 1;   // its bonds u, m (A), n, v (B)
    size_t off_net = 0;              // network tensors and layout scratch
    size_t mps_bytes = 0;            // workspace of the factor construction
    int mixed = 0;                   // sites of general local dimension (explicit form only)
    MixedDesc md;                    // their regrouping
    int nblk = 1;                    // reduction blocks per probe vector
    int64_t nst1 = 1, nst2 = 1;      // bricks along the reduction index of contraction 1, 2
    // workspace carve-up (byte offsets)
    size_t off_Paeb = 0, off_Pbea = 0, off_Xt = 0, off_Ups = 0, off_Ypart = 0, off_U1part = 0;
    size_t off_P1s = 0, off_P2s = 0, off_Up = 0, off_U2 = 0, off_Xs = 0;
    size_t off_Pabe = 0, off_Pabc = 0, off_Cd = 0, off_rho = 0;
    size_t off_Xq = 0, off_Ym = 0;
    size_t off_mps = 0, off_Z1 = 0, off_Z2 = 0, off_Z2p = 0, off_Z3 = 0, off_nrm = 0;
    size_t off_P32 = 0, off_Q32 = 0, off_X32 = 0;   // complex64 copies (FP32 factorised operator)
    size_t off_Q = 0, off_w = 0, off_alpha = 0, off_beta = 0, off_F = 0, off_G = 0;
    size_t off_stats = 0, off_red = 0, off_h = 0, off_steps = 0, off_fit = 0, off_feat = 0, off_mlp = 0;
    size_t off_chk = 0;              // the state check's partial sums
    size_t total = 0;
    int nQ = 3;                      // Lanczos vector slots
};

// ------------------------------------------------------------ layout
// Zero `bytes` bytes at p (16-byte aligned) with a fill kernel on st.
hipError_t launch_zero(void *p, size_t bytes, hipStream_t st);

// ||psi||^2 and the count of non-finite amplitudes of the D-element state, at
// scratch[2 STATE_CHECK_BLOCKS] and scratch[2 STATE_CHECK_BLOCKS + 1]
// (scratch: STATE_CHECK_BYTES of device memory).
constexpr int STATE_CHECK_BLOCKS = 1024;
constexpr size_t STATE_CHECK_BYTES = (2 * STATE_CHECK_BLOCKS + 2) * sizeof(double);
hipError_t launch_state_check(int dtype, const void *psi, int64_t D, double *scratch, hipStream_t st);

struct PermDesc {
    int L;
    int map[TNSLQ_MAX_QUBITS];   // output bit t <- input bit map[t]
};
// Regroup psi into an R x Kr brick operand (output flat index r * Kr + l),
// writing every brick entry including the zero padding.
hipError_t launch_permute(int prec, int dtype, const void *psi, void *out, int64_t R, int64_t Kr,
                          const PermDesc &pd, int conj, hipStream_t st);

// Explicit rho^{T_B} (intermediary (iii) of Sec. V) from the dense product
// C[i][j] = rho_AB[i][j] (n x n, row-major, accumulator type: FP64 when
// accfp64, else FP32), index (a, b) = a d_B + b:
//   rho^{T_B}[(a, b)][(a', b')] = C[(a, b')][(a', b)].
// As an n x n brick operand of precision `prec` (reduction padding zeroed):
hipError_t launch_pt_bricks(int prec, int accfp64, const void *C, int64_t n, int64_t dB, void *rho, int64_t rho_nst,
                            hipStream_t st);
// As a dense complex128 row-major matrix (from an FP64 product):
hipError_t launch_pt_dense(const double2 *C, int64_t n, int64_t dB, double2 *out, hipStream_t st);

// P[(a, b)][c] of d_A d_B rows and d_E reduction terms as a brick operand
// (conjugated if asked), zeros in the padding.
hipError_t launch_permute_mixed(int prec, int dtype, const void *psi, void *out, const MixedDesc &md, int conj,
                                hipStream_t st);

// ------------------------------------------------------------ Lanczos etc.
struct LzDims {
    int64_t dA, dB, n;   // n = dA * dB per probe
    int K, m, nblk;
};
// Xt arguments below are the brick operand of K d_B rows (k, b') by d_A
// reduction terms a', with xt_nst = brick_stages(prec, d_A).
hipError_t launch_probe_init(int prec, const LzDims &z, uint64_t seed, uint64_t offset, int swapped,
                             double2 *q, void *Xt, int64_t xt_nst, double *alpha, double *beta,
                             hipStream_t st);
hipError_t launch_passA(int accfp64, const LzDims &z, const void *part, int S, int64_t split_stride,
                        int k0, int kc, const double2 *q_prev, const double2 *q_cur, double2 *w,
                        const double *alpha, const double *beta, int j, double *dotpart,
                        hipStream_t st);
hipError_t launch_passB(const LzDims &z, const double *dotpart, const double2 *q_cur, double2 *w,
                        double *alpha, const double *beta, int j, double *nrmpart, int want_norm,
                        hipStream_t st);
hipError_t launch_reorth(const LzDims &z, const double2 *Q, int nvec, int64_t q_slot_stride,
                         double2 *w, double *hpart, double2 *h, const double *alpha,
                         const double *beta, int j, double *nrmpart, hipStream_t st);
hipError_t launch_passC(int prec, const LzDims &z, const double *nrmpart, const double2 *w,
                        double2 *q_next, void *Xt, int64_t xt_nst, const double *alpha,
                        double *beta, int j, hipStream_t st);
// fn: TNSLQ_F_ABS, TNSLQ_F_ENTROPY or TNSLQ_F_PURITY
hipError_t launch_quadrature(const double *alpha, const double *beta, const int *steps, int K,
                             int m, int jlo, int jhi, int fn, double *F, hipStream_t st);
hipError_t launch_steps(const double *alpha, const double *beta, int K, int m, int jdone,
                        int *steps, hipStream_t st);
hipError_t launch_stats(const double *beta, const double *F, int K, int m, int j, double *G,
                        double *stats, hipStream_t st);
// Exponential-fit estimate of every probe after step j (FIT_MIN_POINTS <= j <= m)
// into finf, fsig (K each), G = beta_1^2 finf (may be NULL) and the block
// statistics out[6] = {T, SE, eps_L, E, dE, SE / (T ln 2)}.
hipError_t launch_fit(const double *alpha, const double *beta, const double *F, int K, int m, int j, double *finf,
                      double *fsig, double *G, double *out, hipStream_t st);
hipError_t launch_reduce_partials(int accfp64, const void *part, int S, int64_t split_stride,
                                  int64_t dA, int64_t dB, int K, int swapped, double2 *Y,
                                  hipStream_t st);
// Sum of the S split partials of the first contraction (n = kc dB dE dB
// elements, accumulator type: FP64 for TNSLQ_FP64, else FP32) into the Ups
// brick operand.
hipError_t launch_partials_to_bricks(int prec, const void *part, int S, int64_t split, int64_t n, int nB, int nE,
                                     void *ups, int64_t ups_nst, hipStream_t st);
hipError_t launch_probes_plain(uint64_t seed, uint64_t offset, int K, int64_t d, double2 *X,
                               hipStream_t st);
hipError_t launch_load_vectors(int prec, const double2 *X, int64_t dA, int64_t dB, int K,
                               int swapped, void *Xt, int64_t xt_nst, hipStream_t st);
hipError_t launch_features(const double *alpha, const double *beta, int K, int m, int n_early,
                           double dAB, double dA, double dB, double dE, float *feat,
                           hipStream_t st);

// ------------------------------------------------------------ entropy
// psi regrouped as an R x C matrix in column panels 512 wide (same dtype,
// interleaved complex), and the sum of S partial arrays of n elements.
hipError_t launch_regroup(int dtype, const void *psi, void *out, int64_t R, int64_t C, const PermDesc &pd,
                          hipStream_t st);
// The column MAC: out(s, v, c) = sum_{i in split s} op(M[i][c]) V(v, i) over
// an R x C panel-layout matrix M (C even, and dividing 512 when below it) for
// vectors v < NV, with vdiv = 2^vsh and odiv = 2^osh,
//   V(v, i)      at V[(v / vdiv) vs1 + (v % vdiv) vs2 + i vsi],
//   out(s, v, c) at out[s osplit + (v / odiv) os1 + (v % odiv) os2 + c osc],
// the R rows cut into S equal splits.
struct ColmacDesc {
    const void *M;
    int64_t R, C;
    const double2 *V;
    int NV;
    int vsh;
    int64_t vs1, vs2, vsi;
    double2 *out;
    int osh;
    int64_t osplit, os1, os2, osc;
    int S;
    int64_t rows_per_split;   // set by the launcher
};
hipError_t launch_colmac(int dtype, int conj, ColmacDesc g, hipStream_t st);
hipError_t launch_sum_splits(const double2 *part, int S, int64_t n, double2 *Z, hipStream_t st);
// U2[(k, b)][(c, b')] = sum_s Up[s][(k, b')][(c, b)] for the streaming
// partial-transpose matvec (K probes, dB = 2^nB, dE = 2^nE).
hipError_t launch_sum_transpose_ups(const double2 *Up, int S, int K, int nB, int nE, double2 *U2, hipStream_t st);
// Xq[(k, b)][a] = xq[k][a dB + b] (K probes, dB = 2^nB), the first streaming
// pass's vectors; and Y[k][a dB + b] = sum_s Yt[s][(k, b)][a], the sum of the
// second pass's split partials.
hipError_t launch_vectors_by_b(const double2 *xq, int K, int64_t dA, int nB, double2 *Xq, hipStream_t st);
hipError_t launch_sum_transpose_y(const double2 *Yt, int S, int K, int64_t dA, int nB, double2 *Y, hipStream_t st);
// Caller vectors into FP64 layout order Xs[k][a dB + b].
hipError_t launch_load_vectors_plain(const double2 *X, int64_t dA, int64_t dB, int K, int swapped, double2 *Xs,
                                     hipStream_t st);

// ------------------------------------------------------------ one-read streaming matvec
// Both contractions over psi regrouped as P[c][a][b] (complex64, E slowest)
// for vectors X[k][a d_B + b] (FP64): nblk partial sums Ypart[s][k][a d_B + b],
// s < nblk, each over a contiguous range of the d_E slabs.  Shapes: d_B = 2,
// K = 1, d_A = 2048 or 4096.
constexpr int FUSED_BLOCKS = 256;
bool pt_fused_supported(int dtype, int64_t dA, int64_t dB, int K, int64_t dE);
hipError_t launch_pt_fused(const void *P, const double2 *X, int64_t dA, int64_t dB, int K, int64_t dE, int nblk,
                           double2 *Ypart, hipStream_t st);

// ------------------------------------------------------------ MPS blocks
// Small FP64 complex linear algebra for the matrix-product-state reduction
// (Sec. VI); all matrices row-major, interleaved complex.
// One transfer step of a traced environment through the site tensor
// M[x][s][y] (cx x p x cy): left, E[x][x'] -> [y][y']; right, E[y][y'] ->
// [x][x']; the result scaled to unit trace.  tmp: cx p cy + cy^2 entries of
// scratch (device).
hipError_t launch_transfer(int left, const double2 *E, const double2 *M, int cx, int p, int cy, double2 *Enew,
                           double2 *tmp, hipStream_t st);
// In-place lower Cholesky factor (A = L L^dagger) of an n x n positive
// semidefinite matrix; a pivot not above 1e-13 of the largest diagonal entry
// leaves its column zero; *fail (device) is set if a pivot is not finite and
// is never cleared here.  dmax: one device double of scratch (calls on one
// stream may share it).
hipError_t launch_cholesky(double2 *A, int n, int *fail, double *dmax, hipStream_t st);
// Transfer matrices of MPS sections, T[(x, x')][y'][y] = sum_s S[x][s][y]
// conj(S[x'][s][y']) (row-major, x^2 y^2 entries), each divided by its trace
// sum_{a, c} T[(a, a)][c][c] (s: one device double of scratch):
//   start: no sites, X (n x n, or the identity when null) absorbed on the
//     left bond: T[(u, u')][z'][z] = X[z][u] conj(X[z'][u']);
//   step: one site M (cz x p x cy) appended (A: x^2 cz p cy scratch entries);
//   absorb_right: the section S Y for Y (cy x cv) (H: x^2 cy cv entries).
hipError_t launch_transfer_start(const double2 *X, int64_t n, double2 *T, double *s, hipStream_t st);
hipError_t launch_transfer_step(const double2 *T, const double2 *M, int64_t x, int64_t cz, int64_t p, int64_t cy,
                                double2 *Tnew, double2 *A, double *s, hipStream_t st);
hipError_t launch_transfer_absorb_right(const double2 *T, const double2 *Y, int64_t x, int64_t cy, int64_t cv,
                                        double2 *Tnew, double2 *H, double *s, hipStream_t st);
// out[b] = in[b] (shape d[0..3]) with out axis j = in axis perm[j], for nb
// tensors one after the other.
hipError_t launch_permute4(const double2 *in, const int64_t d[4], const int perm[4], double2 *out, hipStream_t st,
                           int64_t nb = 1);
hipError_t launch_permute4(const float2 *in, const int64_t d[4], const int perm[4], float2 *out, hipStream_t st,
                           int64_t nb = 1);
// out = the n x n identity.
hipError_t launch_identity(double2 *out, int64_t n, hipStream_t st);
// s[0] = sum_{a < x, c < y} Re T[a][a][c][c] (T of shape x, x, y, y).
hipError_t launch_trace_pairs(const double2 *T, int64_t x, int64_t y, double *s, hipStream_t st);
// x *= 1 / sqrt(s[0]) (s on the device).
hipError_t launch_scale_rsqrt(double2 *x, int64_t n, const double *s, hipStream_t st);
// C[b] = op(A[b]) op(B[b]) (with sub: C[b] -= op(A[b]) op(B[b])), op 0 = as
// stored, 1 = transpose, 2 = conjugate transpose (supported pairs: (0,0),
// (1,0), (2,0), (0,2)); op(A) is M x K.  With ks > 1 the reduction is split
// in ks ranges and split s writes its partial product to C[b] + s csk (not
// with sub); batch * ks <= 65535.
hipError_t launch_zgemm(int opa, int opb, const double2 *A, const double2 *B, double2 *C, int M, int N, int K,
                        int64_t lda, int64_t ldb, int64_t ldc, int batch, int64_t sa, int64_t sb, int64_t sc,
                        hipStream_t st, int sub = 0, int ks = 1, int64_t csk = 0);
// The same in FP32 (complex64 operands, FP32 matrix instructions).
hipError_t launch_zgemm(int opa, int opb, const float2 *A, const float2 *B, float2 *C, int M, int N, int K,
                        int64_t lda, int64_t ldb, int64_t ldc, int batch, int64_t sa, int64_t sb, int64_t sc,
                        hipStream_t st, int sub = 0, int ks = 1, int64_t csk = 0);
// out[i] = complex64(in[i]), n entries.
// C[b] = A[b] B[b] (both as stored) written with an exchange: output (r, c),
// r = (r1, r2) with r2 < xm and c = (c1, c2) with c2 < xv, lands at
// ((r1 xm + c1) xm + r2) xv + c2 of C[b] (M a multiple of xm, N of xv,
// M <= 65535 * 64 rows, batch <= 65535).
hipError_t launch_zgemm_xc(const double2 *A, const double2 *B, double2 *C, int M, int N, int K, int64_t lda,
                           int64_t ldb, int batch, int64_t sa, int64_t sb, int64_t sc, int64_t xm, int64_t xv,
                           hipStream_t st);
hipError_t launch_zgemm_xc(const float2 *A, const float2 *B, float2 *C, int M, int N, int K, int64_t lda,
                           int64_t ldb, int batch, int64_t sa, int64_t sb, int64_t sc, int64_t xm, int64_t xv,
                           hipStream_t st);
hipError_t launch_to_c64(const double2 *in, int64_t n, float2 *out, hipStream_t st);
// out[b][j][i][k] = (conj) in[b][i][j][k], nb tensors of shape (n0, n1, n2).
hipError_t launch_swap01(const double2 *in, int64_t nb, int64_t n0, int64_t n1, int64_t n2, int conj, double2 *out,
                         hipStream_t st);
// launch_swap01 without conjugation, and for complex64 tensors.
inline hipError_t launch_swap01(const double2 *in, int64_t nb, int64_t n0, int64_t n1, int64_t n2, double2 *out,
                                hipStream_t st) {
    return launch_swap01(in, nb, n0, n1, n2, 0, out, st);
}
hipError_t launch_swap01(const float2 *in, int64_t nb, int64_t n0, int64_t n1, int64_t n2, float2 *out,
                         hipStream_t st);
// part[256] = sum of |x|^2 over all n entries (partials in part[0..255]).
hipError_t launch_sumsq(const double2 *x, int64_t n, double *part, hipStream_t st);
// Normalisation of a two-factor state psi = P Q: with Ahat = P^dagger P and
// C = Q Q^dagger (both mm entries, the same index order), nrm[0] =
// Re sum Ahat conj(C) = ||psi||^2, and the np entries of P are divided by its
// square root.
hipError_t launch_normalise_factor(const double2 *Ahat, const double2 *C, int64_t mm, double *nrm, double2 *P,
                                   int64_t np, hipStream_t st);
// psi[(a, b, e)] (dA2 x dB2 x dE2, zero padded) = T[(a, u)][w][(b, v)] /
// sqrt(*sumsq), e = (u W + w) V + v.
hipError_t launch_assemble(const double2 *T, int64_t kA, int64_t U, int64_t W, int64_t kB, int64_t V, int64_t dA2,
                           int64_t dB2, int64_t dE2, const double *sumsq, double2 *psi, hipStream_t st);

// ------------------------------------------------------------ MLP
size_t mlp_ws_bytes(int batch);
hipError_t mlp_forward(const float *params, const float *norm, const float *x, int batch, float *out,
                       void *ws, hipStream_t st);
hipError_t mlp_loss_grad(const float *params, const float *norm, const float *x, const float *r,
                         const int *idx, int batch, float *loss, float *grad, void *ws,
                         hipStream_t st);
hipError_t mlp_adam(float *params, float *m, float *v, const float *grad, int n, int t, float lr,
                    hipStream_t st);

}  // namespace tnslq
