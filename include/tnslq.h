/*
 * tnslq.h -- C ABI of libtnslq: tensor-network stochastic Lanczos quadrature
 * (TNSLQ) for the logarithmic negativity of a densely represented pure state,
 * on AMD Instinct MI355X (gfx950).
 *
 * Problem statement (Gray, "Fast Computation of Many-Body Entanglement"):
 *   given a pure state psi of L qubits and two disjoint qubit sets A and B
 *   (the environment C = E is every other qubit), estimate
 *       E(rho_AB) = log2 || rho_AB^{T_B} ||_Tr = log2 Tr | rho_AB^{T_B} |
 *   (Sec. II Eq. 1 and Sec. III Eq. 2) with stochastic Lanczos quadrature
 *   (Sec. III, Algorithm 1), acting with rho_AB^{T_B} lazily through two
 *   contractions against psi (Sec. V Eq. 4, intermediary (i)), and report the
 *   error on the mean (Sec. VIII).
 *
 * Conventions shared by every entry point
 *   - Qubit 0 is the most significant bit of psi's flat index.
 *   - A and B are listed in the order that defines the composite indices a and
 *     b: the first listed qubit is the most significant bit.  An element of a
 *     vector on AB has flat index a * d_B + b.
 *   - Complex data are interleaved (re, im): TNSLQ_C64 = 2 x float,
 *     TNSLQ_C128 = 2 x double.
 *   - Device pointers ("dev") are HIP device allocations owned by the caller;
 *     host pointers ("host") are ordinary host memory owned by the caller.
 *     The library allocates no device memory and keeps none between calls:
 *     every scratch buffer lives in the caller's workspace.
 *   - `stream` is a hipStream_t (NULL = the null stream).  All device work is
 *     ordered on it.  Calls that fill host outputs synchronise that stream
 *     before returning; calls without host outputs return without waiting.
 *   - Errors: every argument is validated before any launch; the call then
 *     returns a negative status and launches nothing.  A failing HIP call
 *     returns TNSLQ_E_DEVICE.  Nothing aborts or throws across the ABI.
 *     tnslq_last_error() gives a one-line description of the last failure on
 *     the calling thread.
 *   - Calls that share one workspace must not overlap in time.
 */
#ifndef TNSLQ_H
#define TNSLQ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- status */
enum {
    TNSLQ_OK = 0,
    TNSLQ_E_ARG = -1,        /* null pointer, size or enum out of range       */
    TNSLQ_E_PARTITION = -2,  /* qubit out of range, repeated, or in A and B    */
    TNSLQ_E_DTYPE = -3,      /* unknown storage type                           */
    TNSLQ_E_WORKSPACE = -4,  /* workspace smaller than the query returned      */
    TNSLQ_E_DEVICE = -5,     /* a HIP runtime call failed                      */
    TNSLQ_E_NONFINITE = -6,  /* psi holds a NaN or infinite amplitude, or the
                                estimate came out NaN or infinite              */
    TNSLQ_E_STATE = -7       /* psi is not normalised: | ||psi||^2 - 1 | above
                                TNSLQ_NORM_TOL_C64 / _C128 for its dtype       */
};

/* The estimates assume a normalised state (Tr rho = 1, Sec. II Eq. 1); a state
 * is checked, never silently renormalised.  tnslq_logneg, tnslq_logneg_dims,
 * tnslq_logneg_surrogate, tnslq_spectral_sum and tnslq_mutual_information
 * read psi once before the Lanczos steps (one synchronisation of the stream)
 * and return TNSLQ_E_NONFINITE for a non-finite amplitude and TNSLQ_E_STATE
 * for a squared norm outside 1 +- the tolerance of its dtype (a complex64
 * state normalised in FP64 and rounded is within 1e-6 of 1).  The block
 * matvecs (tnslq_ptmatvec*) apply Eq. 4 to any psi without a check. */
#define TNSLQ_NORM_TOL_C64 1e-4
#define TNSLQ_NORM_TOL_C128 1e-9

/* State storage. */
enum { TNSLQ_C64 = 0, TNSLQ_C128 = 1 };

/* Arithmetic of the two contractions (Sec. V Eq. 4) on the matrix cores.  The
 * Lanczos recurrence, reorthogonalisation, tridiagonal eigensolve and
 * statistics are FP64 in every mode.  With K d_B <= 8 (d_B the smaller side)
 * the contractions are bound by HBM, not by arithmetic, and run instead as two
 * streaming passes over psi in its own dtype with FP64 products and sums,
 * whatever the precision (tnslq_result.streamed).
 *   FP64    complex FP64 products and sums.
 *   FP32    complex FP32 products, FP32 sums in blocks, blocks summed in FP64.
 *   BF16X3  each FP32 operand split as hi + lo (two BF16 values); products
 *           hi*hi + hi*lo + lo*hi on BF16 matrix cores with FP32 accumulation,
 *           three real products per complex product (the operands also carry
 *           the split of Re + Im, 12 bytes per complex value).
 *   BF16X6  hi + mid + lo split, six BF16 products per real product.        */
enum { TNSLQ_FP64 = 0, TNSLQ_FP32 = 1, TNSLQ_BF16X3 = 2, TNSLQ_BF16X6 = 3 };

#define TNSLQ_MAX_QUBITS 36
#define TNSLQ_MAX_STEPS 128

/* Forms of the operator rho_AB^{T_B} (tnslq_options.operator_form).  Sec. V
 * lists three intermediaries for (rho^{T_B} phi)_{ab}; the subsystem sizes
 * decide which is cheapest.
 *   TNSLQ_OPERATOR_LAZY      intermediary (i) (or (ii), by exchanging the
 *                            roles of A and B): every matvec contracts psi,
 *                            16 D min(d_A, d_B) flops per vector.
 *   TNSLQ_OPERATOR_EXPLICIT  intermediary (iii): rho^{T_B} is formed once as a
 *                            d_A d_B x d_A d_B matrix (8 (d_A d_B)^2 d_E
 *                            flops, rho = P P^dagger with P = psi regrouped as
 *                            (A B) x E, then B's indices exchanged), and every
 *                            matvec is a dense product, 8 (d_A d_B)^2 flops
 *                            per vector.  Needs the matrix in the workspace
 *                            (at most 4 GiB of it).
 *   TNSLQ_OPERATOR_AUTO      the explicit form when it fits and its padded
 *                            flop count over n_steps matvecs is the smaller,
 *                            else the lazy form (always lazy when K d_B <= 8,
 *                            the streaming regime).
 * In the streaming regime the lazy form reads psi once per matvec where that
 * is faster (complex64 psi, at least 256 environment slabs, one vector,
 * d_B = 2 and d_A = 2048 or 4096: each block keeps its share of the result on
 * chip), else in two passes.
 *   TNSLQ_OPERATOR_LAZY_TWO_PASS  the lazy form with the two-pass streaming
 *                            form always (for comparison; the results agree
 *                            to FP64 rounding). */
enum { TNSLQ_OPERATOR_AUTO = 0, TNSLQ_OPERATOR_LAZY = 1, TNSLQ_OPERATOR_EXPLICIT = 2,
       TNSLQ_OPERATOR_LAZY_TWO_PASS = 3 };

/* Stopping rules of tnslq_options.stop_rule. */
enum { TNSLQ_STOP_DIFF = 0, TNSLQ_STOP_FIT = 1 };
#define TNSLQ_FIT_WINDOW 8
#define TNSLQ_FIT_MIN_POINTS 5

/* Subsystems A and B (Sec. V: group psi's indices into A, B and C).  `a` and
 * `b` are host arrays of qubit indices in [0, n_qubits), pairwise distinct and
 * disjoint.  n_a == 0 or n_b == 0 is allowed: the negativity is then exactly 0
 * and no device work is done. */
typedef struct {
    int n_qubits;
    const int *a;
    int n_a;
    const int *b;
    int n_b;
} tnslq_partition;

/* Algorithm 1's inputs (Sec. III): N = n_probes repeats, K_max = n_steps.
 *   reorth       0: the three-vector recurrence of Algorithm 1;
 *                1: full reorthogonalisation (classical Gram-Schmidt, twice)
 *                   against every earlier Lanczos vector of the same probe.
 *   precision    TNSLQ_FP64 ... TNSLQ_BF16X6.
 *   seed, probe_offset
 *                probe k uses SplitMix64 outputs (probe_offset + k) * d_A d_B + i
 *                of the generator seeded with `seed`; element i takes
 *                1j ** (output >> 62).  Runs with disjoint offsets are
 *                independent Hutchinson samples and can be merged.
 *   stop_tol     0: run exactly n_steps steps.  > 0: stop at the first step j
 *                whose estimate E_j and combined error e_j meet
 *                e_j <= stop_tol * max(|E_j|, 1) (the "target precision" of
 *                Sec. VII.B / Sec. VIII, relative, in bits), where e_j depends
 *                on stop_rule.
 *   stop_rule    TNSLQ_STOP_DIFF: E_j from the quadrature of T_j, checked from
 *                j >= 6 with e_j = sqrt(dE^2 + (E_j - E_{j-5})^2), dE the
 *                Hutchinson error of the mean.
 *                TNSLQ_STOP_FIT: Algorithm 1's lanczos_estimate by the
 *                exponential fit of Sec. III.  After step
 *                j >= TNSLQ_FIT_MIN_POINTS + 1 each probe's quadrature values
 *                F_{max(2, j-TNSLQ_FIT_WINDOW+1)..j} (F_1, the one-node rule, is
 *                never fitted) are fitted by least squares with F_inf + a r^t,
 *                r in [-0.99, 0.99] (t = 0 at the window's first point);
 *                G_n = ||phi_n||^2 F_inf,n, sigma_n its uncertainty from the
 *                fit's linearised covariance (0 after a breakdown).
 *                E_j = log2 mean G_n and e_j = sqrt(SE^2 + eps_L^2) / (T ln 2)
 *                with SE the Hutchinson error of the mean T and eps_L the mean
 *                of ||phi_n||^2 sigma_n.  The result is the fitted estimate,
 *                also with stop_tol = 0 (then after n_steps steps, which must
 *                be > TNSLQ_FIT_MIN_POINTS).  With stop_tol > 0 and no step
 *                meeting the target, the result is the plain estimate of the
 *                last step (G_n = ||phi_n||^2 F_{n_steps},n), lanczos_err the
 *                fit's eps_L / (T ln 2) at that step.
 *   operator_form
 *                how rho^{T_B} is applied (TNSLQ_OPERATOR_*, above).
 *   max_probes   0 or <= n_probes: one block of n_probes probes, as above.
 *                > n_probes (needs stop_rule = TNSLQ_STOP_FIT and
 *                stop_tol > 0): Algorithm 1's outer loop over probes, in
 *                blocks of n_probes.  Block b uses probe offsets
 *                probe_offset + b n_probes and runs Lanczos steps until its
 *                own Lanczos error meets the target (lanczos_converged:
 *                eps_L / (T ln 2) <= stop_tol max(|E|, 1) on the block's
 *                fitted estimate, checked from step TNSLQ_FIT_MIN_POINTS + 1,
 *                else n_steps); its fitted G_n and sigma_n join those of the
 *                earlier blocks.  Blocks are added until the estimate over all
 *                probes so far meets the combined target of stop_rule
 *                TNSLQ_STOP_FIT (hutchinson_converged) or the next block would
 *                pass max_probes.  psi is regrouped once.  Only G_host (room
 *                for max_probes values, filled for the probes used) may be
 *                non-NULL among the optional outputs.
 *   chunk_probes 0: the lazy form on the matrix cores contracts as many
 *                probes per launch as fit an intermediary of 2^31 values
 *                (Sec. V Eq. 4, intermediary (i): d_B x d_E d_B values per
 *                probe; 8, 12 or 16 bytes each in FP32, split BF16, FP64).
 *                > 0: at most this many probes per launch.  Either way the
 *                count is rounded up so that every chunk starts on a block of
 *                128 rows (k, b') (a multiple of 128 / d_B when d_B < 128) and
 *                capped at n_probes; the last chunk takes the remainder.  The
 *                estimate does not depend on it; the workspace shrinks with
 *                it.  Ignored by the streaming, explicit and MPS forms.
 */
typedef struct {
    int n_probes;
    int n_steps;
    int reorth;
    int precision;
    uint64_t seed;
    uint64_t probe_offset;
    double stop_tol;
    int stop_rule;
    int operator_form;      /* TNSLQ_OPERATOR_AUTO / _LAZY / _EXPLICIT        */
    int max_probes;         /* > n_probes: Algorithm 1's loop over probes     */
    int chunk_probes;       /* 0, or the most probes per contraction launch   */
} tnslq_options;

typedef struct {
    double logneg;          /* log2 of the mean of G_n                        */
    double logneg_se;       /* trace_norm_se / (trace_norm ln 2); NaN if N = 1 */
    double trace_norm;      /* mean of G_n = ||phi_n||^2 F_{m} (TNSLQ_STOP_FIT:
                               ||phi_n||^2 F_inf,n, unless a target was set and
                               never met)                                     */
    double trace_norm_se;   /* sqrt(Var(G) / N), sample variance (N - 1)       */
    int steps_done;         /* Lanczos steps run on the probe block            */
    int steps_min;          /* fewest steps of any probe (breakdown stops one) */
    int swapped_ab;         /* 1 if the roles of A and B were exchanged so that
                               the transposed side is the smaller one          */
    int n_matvecs;          /* block matvecs performed                          */
    int n_contract_launches;/* launches of each contraction kernel             */
    double t_layout_ms;     /* psi regrouping + operand preparation (device)   */
    double t_matvec_ms;     /* both contractions + split-K merge (device)      */
    double t_contract1_ms;  /* first contraction (over a'), all launches       */
    double t_contract2_ms;  /* second contraction (over b', c), all launches   */
    double t_lanczos_ms;    /* recurrence, reorthogonalisation (device)        */
    double t_total_ms;      /* whole call, host clock                          */
    double lanczos_err;     /* Lanczos part of the error of logneg, in bits:
                               |E_j - E_{j-5}| (TNSLQ_STOP_DIFF, NaN for j < 6)
                               or eps_L / (T ln 2) (TNSLQ_STOP_FIT)            */
    int streamed;           /* 0 if the contractions ran on the matrix cores
                               in `precision`; in the streaming regime (K d_B
                               <= 8 after the role choice, FP64 arithmetic) 1
                               for two passes over psi, 2 for one read        */
    int explicit_operator;  /* 1 if rho^{T_B} was formed explicitly
                               (intermediary (iii)); the roles of A and B are
                               then never exchanged, t_contract1_ms is 0 and
                               t_contract2_ms times the dense products; the
                               forming is part of t_layout_ms                  */
    int n_probes_used;      /* probes behind the estimate (n_probes, or a
                               multiple of it with max_probes)                 */
    int mps_matvec;         /* tnslq_logneg_mps: the matvec that ran,
                               TNSLQ_MPS_MATVEC_FACTORS or _NETWORK; else 0    */
} tnslq_result;

/* ------------------------------------------------------------ utilities */
const char *tnslq_status_str(int status);
/* Description of the last failure on the calling thread ("" if none). */
const char *tnslq_last_error(void);
/* ABI version, currently 4. */
int tnslq_version(void);

/* -------------------------------------------------- logarithmic negativity */

/* Bytes of device workspace tnslq_logneg needs for this problem (host call,
 * no device work).  Writes *bytes; returns a status. */
int tnslq_workspace_bytes(int dtype, const tnslq_partition *part, const tnslq_options *opt,
                          size_t *bytes);

/* SLQ estimate of E(rho_AB) (Sec. III Algorithm 1 with the lazy operator of
 * Sec. V Eq. 4).
 *   psi_dev    device, 2^n_qubits complex elements of `dtype`, read only.
 *   ws_dev     device workspace of at least tnslq_workspace_bytes() bytes,
 *              256-byte aligned; contents on entry are ignored.
 *   res        host, filled on success.
 * Optional host outputs (NULL to skip), with N = n_probes, m = n_steps:
 *   G_host     N doubles: the per-probe estimates G_n.
 *   alpha_host N*m doubles, row n = alpha_1..alpha_m of probe n (0 past a stop).
 *   beta_host  N*(m+1) doubles, row n = beta_1 (= ||phi_n||) .. beta_{m+1}.
 *   F_host     N*m doubles, row n = F_1..F_m (Algorithm 1's quadrature values
 *              for the normalised probe; values past a stop repeat the last).
 *   steps_host N ints: Lanczos steps each probe ran before stopping.
 * A probe stops early (Lanczos breakdown, not an error) when
 * beta_{j+1} <= 1e-12 * (max_{i<=j} |alpha_i| + max_{2<=i<=j} beta_i); its
 * quadrature is then exact.  Synchronises `stream`. */
int tnslq_logneg(const void *psi_dev, int dtype, const tnslq_partition *part,
                 const tnslq_options *opt, void *ws_dev, size_t ws_bytes, void *stream,
                 tnslq_result *res, double *G_host, double *alpha_host, double *beta_host,
                 double *F_host, int *steps_host);

/* ------------------------------------------ sites of any local dimension */

/* Subsystems of a state on sites of general local dimension (the paper's
 * method is stated for any d_A, d_B, d_C; Sec. V).  psi's flat index is in
 * mixed radix over sites 0 .. n_sites-1 with site 0 most significant and
 * dims[s] >= 2 values at site s (the product at most 2^40).  `a` and `b` list
 * sites, pairwise distinct and disjoint; C is the other sites in increasing
 * order.  Index (a, b) of A B runs over A's sites in the order given, then
 * B's, b fastest. */
typedef struct {
    int n_sites;
    const int *dims;
    const int *a;
    int n_a;
    const int *b;
    int n_b;
} tnslq_partition_dims;

/* tnslq_workspace_bytes / tnslq_logneg for such sites.  They use the explicit
 * operator only (operator_form TNSLQ_OPERATOR_AUTO or _EXPLICIT; _LAZY is an
 * argument error), so d_A d_B <= 16384; everything else, including the probe
 * law (element i of probe k from output (probe_offset + k) d_A d_B + i) and
 * the optional outputs, is as for qubits. */
int tnslq_workspace_bytes_dims(int dtype, const tnslq_partition_dims *part, const tnslq_options *opt,
                               size_t *bytes);
int tnslq_logneg_dims(const void *psi_dev, int dtype, const tnslq_partition_dims *part, const tnslq_options *opt,
                      void *ws_dev, size_t ws_bytes, void *stream, tnslq_result *res, double *G_host,
                      double *alpha_host, double *beta_host, double *F_host, int *steps_host);

/* ----------------------------------------- matrix product states (Sec. VI) */

/* A matrix product state (Eq. 5, Fig. 4): site i holds a complex128 tensor
 * M_i[x][s][y] of shape (bond[i], phys[i], bond[i+1]), row-major, the sites'
 * tensors one after the other in `tensors` (device, read only).
 *   open boundaries (bond[0] = bond[n] = 1): psi_{s_0 .. s_{L-1}} =
 *     M_0[0][s_0][:] M_1[:][s_1][:] ... M_{L-1}[:][s_{L-1}][0];
 *   periodic boundaries (bond[0] = bond[n] > 1, a ring): psi_{s_0 .. s_{L-1}}
 *     = Tr M_0[:][s_0][:] ... M_{L-1}[:][s_{L-1}][:] (the closing bond summed);
 * site 0 most significant.  The state need not be normalised.
 * `sections` chooses how the matrices of compressed sections (below) are
 * formed:
 *   TNSLQ_MPS_SECTIONS_EXPLICIT: the section is contracted over its whole
 *     physical index (p^len x bond^2 entries, at most 2^31) and its Gram
 *     matrix is a product over that index;
 *   TNSLQ_MPS_SECTIONS_TRANSFER: its transfer matrix T[(x, x')][y'][y] =
 *     sum_s S[x][s][y] conj(S[x'][s][y']) is built one site at a time (the
 *     first step of Sec. VI's lateral compression; bond^4 entries, about
 *     2 bond^5 p complex multiply-adds per site), so sections of any length
 *     are reached; the Gram and trace matrices are T with its axes regrouped;
 *   TNSLQ_MPS_SECTIONS_AUTO (0): per section, the cheaper of the two by that
 *     count, the transfer route whenever the explicit section would exceed
 *     2^26 entries.
 * Both give the same effective state up to rounding. */
#define TNSLQ_MPS_SECTIONS_AUTO 0
#define TNSLQ_MPS_SECTIONS_EXPLICIT 1
#define TNSLQ_MPS_SECTIONS_TRANSFER 2
/* `matvec` chooses how tnslq_logneg_mps contracts a probe through the
 * compressed operator (below); both apply the same operator:
 *   TNSLQ_MPS_MATVEC_FACTORS: psi_eff's two factors P, Q (four products);
 *   TNSLQ_MPS_MATVEC_NETWORK: the blocks' R_A, R_B and the traced gap's and
 *     ring's matrices E_W, E_Z kept apart (six products, every intermediate
 *     at most bond^4 per probe, as the network of Sec. VI);
 *   TNSLQ_MPS_MATVEC_AUTO (0): the one with fewer multiply-adds per probe
 *     (the factors on ties).
 * tnslq_mps_effective_state ignores it. */
#define TNSLQ_MPS_MATVEC_AUTO 0
#define TNSLQ_MPS_MATVEC_FACTORS 1
#define TNSLQ_MPS_MATVEC_NETWORK 2
typedef struct {
    int n_sites;
    const int *phys;        /* host, n_sites entries >= 2                        */
    const int *bond;        /* host, n_sites + 1 entries in [1, 4096],
                               bond[0] = bond[n]                                 */
    const void *tensors;    /* device, complex128                                */
    int sections;           /* TNSLQ_MPS_SECTIONS_*                              */
    int matvec;             /* TNSLQ_MPS_MATVEC_*                                */
} tnslq_mps;

/* Contiguous blocks A = sites [a0, a0 + n_a) and B = [b0, b0 + n_b), a0 + n_a
 * <= b0; bonds u enters A, m leaves it, n enters B, v leaves it.  Sec. VI's
 * compressed form of rho_AB^{T_B}, reduced to a dense effective state psi_eff
 * with the same nonzero spectrum of the partial transpose (so the same trace
 * norm), normalised:
 *   - open chain: the sites left of A and right of B are traced; their
 *     transfer products E_L, E_R (positive, on u and v) are factored
 *     E = X X^dagger (Cholesky) and absorbed into A and B, whose outer bond
 *     indices u, v become traced environment indices;
 *   - ring: the sites right of B and left of A form one outer section
 *     O[v][o][u] through the closing bond (the identity delta(v, u) when the
 *     blocks cover the ring); it is traced: Z[v][u][z] with Z Z^dagger its
 *     transfer matrix grouped as (v, u) against (v', u') (Cholesky when its
 *     physical space is larger than v u, else O itself), z joining the
 *     environment;
 *   - vertical decomposition: a block whose physical space is larger than its
 *     two bonds' (p^{n_a} > bond[a0] bond[a0 + n_a]) is replaced by R with
 *     R^dagger R its Gram matrix over the physical index (Cholesky): an
 *     isometry on the block's space, which keeps the nonzero spectrum of the
 *     partial transpose; effective dimension <= bond^2;
 *   - the gap between A and B (if any) is traced like the outer section:
 *     W[m][n][w], W W^dagger its transfer matrix grouped as (m, n) against
 *     (m', n').
 * E' = (u, w, v) on an open chain, (w, z) on a ring.  psi_eff's parts A', B',
 * E' are each zero padded to a power of two, 2^q_A, 2^q_B, 2^q_E, so that
 * tnslq_logneg (qubits: A = [0, q_A), B = [q_A, q_A + q_B)) applies to it
 * unchanged; the padding adds only zero eigenvalues.  Factored matrices are
 * at most 16384 wide (bond[a0] bond[a0 + n_a] and its like for compressed
 * sections).
 *   tnslq_mps_effective_state_size: q[3] = (q_A, q_B, q_E) and the workspace
 *     bytes (host only).
 *   tnslq_mps_effective_state: writes psi_eff, 2^(q_A + q_B + q_E) complex128
 *     (device), A' most significant.  The factorisations are Cholesky factors
 *     of positive semidefinite matrices: where a matrix is rank deficient (a
 *     pivot at most 1e-13 of its largest diagonal entry) the column is left
 *     zero, which only adds zero padding to psi_eff.  Returns
 *     TNSLQ_E_NONFINITE if a factored matrix holds non-finite values.
 *     Synchronises `stream` (to read that outcome). */
int tnslq_mps_effective_state_size(const tnslq_mps *mps, int a0, int n_a, int b0, int n_b, int *q,
                                   size_t *ws_bytes);
int tnslq_mps_effective_state(const tnslq_mps *mps, int a0, int n_a, int b0, int n_b, void *psi_dev, void *ws_dev,
                              size_t ws_bytes, void *stream);

/* Algorithm 1 on the same two blocks without forming psi_eff (Sec. VI: the
 * operator as a small tensor network).  With the factors above, psi_eff has
 * the form psi[a][b][(u', v)] = sum_m P[a][u'][m] Q[b][m][v] (open chain,
 * adjacent blocks: P = R_A and m the bond between them; with a gap: P = R_A W,
 * u' = (u, w), m the bond entering B; ring: P = R_A W with u' = w and
 * m = (n, u), Q = R_B Z with v = z), and each matvec is four complex products,
 *   Z1 = P^dagger X,  Z2 = Z1 Q,  Z3 = P Z2 (m and m' exchanged),
 *   Y[a][b] = sum_{m', v} Z3[a][(m', v)] conj Q[b][(m', v)],
 * about 2 k chi^4 + 2 k^2 chi^2 complex multiply-adds per probe for
 * k = d_A' = d_B' and bonds chi on an open chain with adjacent blocks,
 * against 2 k^3 chi^2 for the lazy form on psi_eff.  Across a gap (u' is
 * chi w wide) and on a ring (m is chi^2 wide) the factors grow; the network
 * form keeps E_W[(m, n), (m', n')] = sum_w W[m][n][w] conj W[m'][n'][w] and
 * E_Z[(v, u), (v', u')] = sum_z Z[v][u][z] conj Z[v'][u'][z] apart:
 *   T1 = R_A^dagger X, T2 = T1 R_B               (T2[u'][m'][n][v]),
 *   T3[m][n'][u'][v] = sum_{m', n} E_W T2        (adjacent: T2 regrouped),
 *   T4[u][v'][m][n'] = sum_{v, u'} E_Z T3        (open chain: T3 regrouped),
 *   Y[a][b] = sum R_A[a][u][m] T4[u][v'][m][n'] conj R_B[b][n'][v'],
 * about 4 k chi^4 + (chi^2)^3 per traced section, every intermediate at
 * most chi^4 entries per probe.  The Lanczos vectors run over (a, b),
 * a d_B' + b, n = d_A' d_B' entries, unpadded; the estimate and every output are those of
 * tnslq_logneg on psi_eff (same probes, same stopping rules, the loop over
 * probes with max_probes).
 *   opt->precision TNSLQ_FP64 (complex products in FP64) or TNSLQ_FP32
 *   (complex64 factors and intermediates on the FP32 matrix instructions;
 *   the Lanczos recurrence stays FP64), and
 *   opt->operator_form TNSLQ_OPERATOR_AUTO; res->streamed and
 *   res->explicit_operator are 0.  Probes are processed in chunks whose
 *   intermediates fit 8 GiB.  Errors as tnslq_logneg, plus those of
 *   tnslq_mps_effective_state; synchronises `stream`. */
int tnslq_workspace_bytes_mps(const tnslq_mps *mps, int a0, int n_a, int b0, int n_b, const tnslq_options *opt,
                              size_t *bytes);
int tnslq_logneg_mps(const tnslq_mps *mps, int a0, int n_a, int b0, int n_b, const tnslq_options *opt, void *ws_dev,
                     size_t ws_bytes, void *stream, tnslq_result *res, double *G_host, double *alpha_host,
                     double *beta_host, double *F_host, int *steps_host);

/* ------------------------------------------------ partial-transpose matvec */

/* Workspace bytes for tnslq_ptmatvec with n_vectors vectors. */
int tnslq_ptmatvec_workspace_bytes(int dtype, const tnslq_partition *part, int n_vectors,
                                   int precision, int chunk_vectors, size_t *bytes);

/* Y = rho_AB^{T_B} X for a block of n_vectors vectors (Sec. V Eq. 4:
 * (rho^{T_B} phi)_{ab} = sum_{a',b',c} psi_{ab'c} psi*_{a'bc} phi_{a'b'}),
 * contracted lazily through intermediary (i) in the given precision.
 *   X_dev  device, n_vectors x (d_A d_B) complex128, row n = vector n.
 *   Y_dev  device, same shape, overwritten (must not alias X_dev).
 *   chunk_vectors  0 or the most vectors per contraction launch on the
 *          matrix cores, rounded as tnslq_options.chunk_probes (the result
 *          does not depend on it).
 * Does not synchronise. */
int tnslq_ptmatvec(const void *psi_dev, int dtype, const tnslq_partition *part, int n_vectors,
                   const void *X_dev, void *Y_dev, int precision, int chunk_vectors, void *ws_dev,
                   size_t ws_bytes, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): tnslq_ptmatvec
 * with the workspace taken from a fixed scratch array the library holds on
 * each GPU (TNSLQ_STATIC_SCRATCH_BYTES, kept from the library's load until
 * the process ends) instead of a caller's buffer.  Arguments, results and
 * errors as tnslq_ptmatvec; the problem must fit the scratch:
 * tnslq_ptmatvec_workspace_bytes() <= TNSLQ_STATIC_SCRATCH_BYTES (a smaller
 * chunk_vectors shrinks it), else TNSLQ_E_WORKSPACE before any device work.
 * The scratch is that of the calling thread's current device, and `stream`
 * must belong to that device.  Calls no allocating routine.  Every call on a
 * GPU uses the same scratch, which keeps the last call's contents (nothing
 * is assumed about them on entry): calls on one GPU whose device work
 * overlaps in time (different streams or threads without ordering between
 * them) race and give undefined results.  Does not synchronise. */
#define TNSLQ_STATIC_SCRATCH_BYTES ((size_t)64 << 20)
int tnslq_ptmatvec_static(const void *psi_dev, int dtype, const tnslq_partition *part, int n_vectors,
                          const void *X_dev, void *Y_dev, int precision, int chunk_vectors, void *stream);

/* ------------------------------------------- explicit partial transpose */

/* Workspace bytes for tnslq_rho_pt. */
int tnslq_rho_pt_workspace_bytes(int dtype, const tnslq_partition *part, size_t *bytes);

/* The partially traced, partially transposed density matrix of Sec. V's
 * intermediary (iii), formed on the device in FP64:
 *   rho_out[(a, b)][(a', b')] = sum_c psi_{a b' c} psi*_{a' b c},
 * rows and columns (a, b) with a = A's qubits in the order given (most
 * significant first), b likewise, b fastest; c runs over the other qubits.
 *   rho_dev  device, (d_A d_B)^2 complex128, row-major, overwritten.
 * At most d_A d_B = 16384.  Needs non-empty A and B.  Does not synchronise. */
int tnslq_rho_pt(const void *psi_dev, int dtype, const tnslq_partition *part, void *rho_dev, void *ws_dev,
                 size_t ws_bytes, void *stream);

/* tnslq_rho_pt for sites of general local dimension (above). */
int tnslq_rho_pt_dims_workspace_bytes(int dtype, const tnslq_partition_dims *part, size_t *bytes);
int tnslq_rho_pt_dims(const void *psi_dev, int dtype, const tnslq_partition_dims *part, void *rho_dev, void *ws_dev,
                      size_t ws_bytes, void *stream);

/* ------------------------------------------- other spectral sums (entropy) */

/* The same stochastic Lanczos quadrature with the partial transpose dropped
 * (the paper's closing section: von Neumann entropy, mutual information and
 * other functions of reduced density matrices).  For a subsystem S of the
 * pure state psi, rho_S = Tr_R |psi><psi| = Psi Psi^dagger with Psi = psi
 * regrouped as a d_S x d_R matrix (S's qubits in the given order, most
 * significant first; R the other qubits in increasing order).  The Krylov
 * space is built on the smaller of S and R (rho_S and rho_R share their
 * non-zero spectrum), and rho is applied lazily, rho X = Psi (Psi^dagger X),
 * by two passes over psi with FP64 products and sums.  The estimate of
 * Tr f(rho) is the Hutchinson mean of G_n = ||phi_n||^2 F_m (no logarithm). */
enum { TNSLQ_F_ABS = 0,       /* f(x) = |x|: the trace norm (tnslq_logneg)   */
       TNSLQ_F_ENTROPY = 1,   /* f(x) = -x log2 x (0 for x <= 0): S in bits */
       TNSLQ_F_PURITY = 2 };  /* f(x) = x^2: Tr rho^2                       */

typedef struct {
    double value;           /* mean of G_n, the estimate of Tr f(rho_S)       */
    double value_se;        /* sqrt(Var(G) / N), sample variance (N - 1)       */
    int steps_done;         /* Lanczos steps run                               */
    int steps_min;          /* fewest steps of any probe (breakdown stops one) */
    int complement;         /* 1 if the Krylov space is that of rho_R          */
    int n_qubits_side;      /* qubits of the side the Krylov space lives on    */
    double t_layout_ms;     /* regrouping psi (device)                         */
    double t_matvec_ms;     /* both passes over psi, all steps (device)        */
    double t_lanczos_ms;    /* recurrence, reorthogonalisation (device)        */
    double t_total_ms;      /* whole call, host clock                          */
} tnslq_spectral_result;

/* Workspace bytes for tnslq_spectral_sum on subsystem s[0..n_s) (host call). */
int tnslq_spectral_workspace_bytes(int dtype, int n_qubits, const int *s, int n_s, const tnslq_options *opt,
                                   size_t *bytes);

/* Tr f(rho_S) by Algorithm 1 with opt->n_probes probes and exactly
 * opt->n_steps Lanczos steps (opt->precision must be TNSLQ_FP64; stop_tol must
 * be 0; reorth, seed and probe_offset as for tnslq_logneg, with d = the side's
 * dimension in place of d_A d_B).  n_s == 0 or n_s == n_qubits is exact
 * without device work (a pure state: entropy 0, purity 1).  Host arrays as
 * for tnslq_logneg, may be NULL.  Synchronises the stream before returning. */
int tnslq_spectral_sum(const void *psi_dev, int dtype, int n_qubits, const int *s, int n_s, int fn,
                       const tnslq_options *opt, void *ws_dev, size_t ws_bytes, void *stream,
                       tnslq_spectral_result *res, double *G_host, double *alpha_host, double *beta_host,
                       double *F_host, int *steps_host);

/* Workspace bytes for tnslq_mutual_information: the largest of its three
 * spectral sums. */
int tnslq_mutual_information_workspace_bytes(int dtype, const tnslq_partition *part,
                                             const tnslq_options *opt, size_t *bytes);

/* Mutual information I(A:B) = S(A) + S(B) - S(AB) of the pure state psi, each
 * entropy by tnslq_spectral_sum (S(AB) through the smaller of AB and E), with
 * the probe offsets probe_offset, +n_probes, +2 n_probes so that the three
 * estimates are independent.  out[8] = {I, I_se, S_A, S_A_se, S_B, S_B_se,
 * S_AB, S_AB_se} (host); the errors of I add in quadrature.  Synchronises the
 * stream before returning. */
int tnslq_mutual_information(const void *psi_dev, int dtype, const tnslq_partition *part,
                             const tnslq_options *opt, void *ws_dev, size_t ws_bytes, void *stream,
                             double *out);

/* ----------------------------------------------------- Gauss quadrature */

/* For each probe n and each k = 1..n_steps, F[n][k-1] = sum_j tau_j^2 |theta_j|
 * where theta_j, w_j are the eigenpairs of T_k = tridiag(alpha_1..alpha_k;
 * beta_2..beta_k) and tau_j the first component of w_j (Sec. III,
 * Algorithm 1's quadrature block), with k capped at steps[n].
 *   alpha_dev  device, n_probes x n_steps doubles.
 *   beta_dev   device, n_probes x (n_steps+1) doubles (beta_1 first).
 *   steps_dev  device, n_probes ints in [1, n_steps].
 *   F_dev      device, n_probes x n_steps doubles, written.
 * Does not synchronise. */
int tnslq_quadrature(const double *alpha_dev, const double *beta_dev, const int *steps_dev,
                     int n_probes, int n_steps, double *F_dev, void *stream);

/* The probe block itself: X[n][i] = 1j ** (SplitMix64(seed) output
 * ((probe_offset + n) * d + i) >> 62), written as complex128 to the device
 * array X_dev (n_probes x d).  Does not synchronise. */
int tnslq_probes(uint64_t seed, uint64_t probe_offset, int n_probes, int64_t d, void *X_dev,
                 void *stream);

/* ------------------------------------------ learned early stopping (MLP) */
/* A 19 -> 256 -> 256 -> 2 perceptron with ReLU (the project's addition; the
 * paper has no learned part).  Parameters are one float array of
 * TNSLQ_MLP_NPARAMS values, W1 (256 x 19, row = output unit), b1, W2 (256 x
 * 256), b2, W3 (2 x 256), b3.  Weights enter every product rounded to BF16
 * (nearest, ties to even); sums are FP32.  `norm` holds 38 floats: the 19
 * feature means then the 19 feature scales; inputs are standardised as
 * (t(x) - mean) / scale, where t is asinh for the 16 Lanczos-coefficient
 * features and the identity for the three log2 sizes.  Output row = (u0, u1):
 * predicted residual mean and log variance. */
#define TNSLQ_MLP_NIN 19
/* Lanczos steps the surrogate may read before deciding. */
#define TNSLQ_SURROGATE_MIN_EARLY 4
#define TNSLQ_SURROGATE_MAX_EARLY 8
#define TNSLQ_MLP_NHID 256
#define TNSLQ_MLP_NOUT 2
#define TNSLQ_MLP_NPARAMS 71426

/* Workspace bytes for a batch of `batch` rows (forward and gradient). */
int tnslq_mlp_workspace_bytes(int batch, size_t *bytes);

/* out_dev[batch x 2] = network(x_dev[batch x 19]).  All pointers device.
 * Does not synchronise. */
int tnslq_mlp_forward(const float *params_dev, const float *norm_dev, const float *x_dev,
                      int batch, float *out_dev, void *ws_dev, size_t ws_bytes, void *stream);

/* Gaussian negative log-likelihood of targets r_dev[batch],
 * L = (1/B) sum 0.5 (u1 + (r - u0)^2 exp(-u1)), and its gradient with
 * respect to the parameters (BF16 rounding treated as the identity).
 * loss_dev: 1 float; grad_dev: TNSLQ_MLP_NPARAMS floats, overwritten.
 * Does not synchronise. */
int tnslq_mlp_loss_grad(const float *params_dev, const float *norm_dev, const float *x_dev,
                        const float *r_dev, int batch, float *loss_dev, float *grad_dev,
                        void *ws_dev, size_t ws_bytes, void *stream);

/* One Adam step (Kingma & Ba) on FP32 master parameters in place, t >= 1,
 * beta1 = 0.9, beta2 = 0.999, eps = 1e-8.  m_dev, v_dev: moment buffers.
 * Does not synchronise. */
int tnslq_mlp_adam(float *params_dev, float *m_dev, float *v_dev, const float *grad_dev, int t,
                   float lr, void *stream);

/* Minibatch training: for s = 0..n_batches-1, gather rows idx_dev[s*batch ..
 * (s+1)*batch) of (x_dev, r_dev), compute the gradient and take Adam step
 * t0 + s.  losses_dev (device, n_batches floats, may be NULL) receives each
 * step's loss.  Does not synchronise. */
int tnslq_mlp_train(float *params_dev, float *m_dev, float *v_dev, const float *norm_dev,
                    const float *x_dev, const float *r_dev, const int *idx_dev, int batch,
                    int n_batches, int t0, float lr, float *losses_dev, void *ws_dev,
                    size_t ws_bytes, void *stream);

/* Early-stopping surrogate run.  Runs `early_steps` Lanczos steps of
 * tnslq_logneg, forms the 19 features (slots 0..7: probe means of d_A d_B
 * alpha_1..early_steps; slots 8..15: probe means of d_A d_B
 * beta_2..early_steps+1; slots past early_steps hold zero; then log2 d_A,
 * log2 d_B, log2 d_E), and evaluates the network: mu = E_early + y_scale *
 * u0, sigma = y_scale * exp(u1 / 2), with E_early the SLQ estimate from
 * T_{early_steps}.  If sigma <= tol * max(|mu|, 1) the result is (mu,
 * sigma); otherwise the same Lanczos state continues to opt->n_steps (the
 * fallback) and the result is full SLQ's.
 *   early_steps  TNSLQ_SURROGATE_MIN_EARLY..TNSLQ_SURROGATE_MAX_EARLY, the
 *                value the network was trained with (its checkpoint records
 *                it).
 *   res          as tnslq_logneg; when the surrogate is accepted, logneg =
 *                mu and logneg_se = sigma.
 *   info_host    host, 5 doubles: mu, sigma, E_early, used_fallback (0/1),
 *                E_full (NaN when not run).
 * Synchronises `stream`. */
int tnslq_logneg_surrogate(const void *psi_dev, int dtype, const tnslq_partition *part,
                           const tnslq_options *opt, const float *params_dev,
                           const float *norm_dev, float y_scale, int early_steps, double tol,
                           void *ws_dev, size_t ws_bytes, void *stream, tnslq_result *res,
                           double *info_host);

#ifdef __cplusplus
}
#endif
#endif /* TNSLQ_H */
