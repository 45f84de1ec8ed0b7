// FP64 Lanczos recurrence, reorthogonalisation, Gauss quadrature and
// Hutchinson statistics (Sec. III, Algorithm 1; Sec. VIII).
//
// Vectors are complex128, one row of d_A d_B elements per probe.  Reductions
// over a vector are done in two fixed-order stages (per-block tree, then a
// sequential sum of the block partials) so that results are bitwise
// reproducible run to run; no floating-point atomics are used.
#include <float.h>

#include "tnslq_internal.h"

namespace tnslq {
namespace {

constexpr double BREAKDOWN_TOL = 1e-12;

// Fixed-order sum over a 256-thread block (wave64 shuffles, then LDS).
__device__ inline double block_sum(double v, double *sh) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0) {
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += sh[i];
        sh[8] = t;
    }
    __syncthreads();
    return sh[8];
}

// Sum of partials[0..cnt) in a fixed order, the same in every block.
__device__ inline double sum_partials(const double *p, int cnt, double *sh) {
    double v = 0.0;
    for (int i = threadIdx.x; i < cnt; i += blockDim.x) v += p[i];
    return block_sum(v, sh);
}

// Step (1-based) at which the probe broke down among steps 1..jmax, or 0.
// Breakdown at step s: beta_{s+1} <= tol * (max_{i<=s} |alpha_i| + max_{2<=i<=s} beta_i).
__device__ inline int first_break(const double *alpha_k, const double *beta_k, int jmax) {
    double amax = 0.0, bmax = 0.0;
    for (int s = 1; s <= jmax; ++s) {
        amax = fmax(amax, fabs(alpha_k[s - 1]));
        if (s >= 2) bmax = fmax(bmax, beta_k[s - 1]);
        if (beta_k[s] <= BREAKDOWN_TOL * (amax + bmax)) return s;
    }
    return 0;
}

__device__ inline void elem_range(int64_t n, int nblk, int64_t &beg, int64_t &end) {
    const int64_t chunk = (n + nblk - 1) / nblk;
    beg = (int64_t)blockIdx.x * chunk;
    end = beg + chunk < n ? beg + chunk : n;
}

// w = Y - beta_j q_{j-1} with Y the sum of the contraction's split partials;
// partial sums of Re<q_j, w>.
template <typename AccT>
__global__ void __launch_bounds__(256) k_passA(const AccT *__restrict__ part, int S, int64_t split_stride,
                                               int k0, int64_t n, const double2 *__restrict__ q_prev,
                                               const double2 *__restrict__ q_cur, double2 *__restrict__ w,
                                               const double *__restrict__ alpha,
                                               const double *__restrict__ beta, int m, int j, int nblk,
                                               double *__restrict__ dotpart) {
    __shared__ double sh[16];
    const int kl = blockIdx.y, k = k0 + kl;
    const double *ak = alpha + (int64_t)k * m;
    const double *bk = beta + (int64_t)k * (m + 1);
    const bool live = first_break(ak, bk, j - 1) == 0;
    const double bj = (j > 1) ? bk[j - 1] : 0.0;
    int64_t beg, end;
    elem_range(n, nblk, beg, end);
    double acc = 0.0;
    const int64_t base = (int64_t)k * n;
    for (int64_t e = beg + threadIdx.x; e < end; e += blockDim.x) {
        double re = 0.0, im = 0.0;
        for (int s = 0; s < S; ++s) {
            AccT v = part[s * split_stride + (int64_t)kl * n + e];
            re += (double)v.x;
            im += (double)v.y;
        }
        if (j > 1) {
            double2 p = q_prev[base + e];
            re -= bj * p.x;
            im -= bj * p.y;
        }
        if (!live) re = im = 0.0;
        w[base + e] = make_double2(re, im);
        double2 q = q_cur[base + e];
        acc += q.x * re + q.y * im;
    }
    acc = block_sum(acc, sh);
    if (threadIdx.x == 0) dotpart[(int64_t)k * nblk + blockIdx.x] = acc;
}

// alpha_j = Re<q_j, w>;  w -= alpha_j q_j;  optional partial sums of |w|^2.
__global__ void __launch_bounds__(256) k_passB(const double *__restrict__ dotpart, int64_t n,
                                               const double2 *__restrict__ q_cur, double2 *__restrict__ w,
                                               double *__restrict__ alpha, const double *__restrict__ beta,
                                               int m, int j, int nblk, double *__restrict__ nrmpart,
                                               int want_norm) {
    __shared__ double sh[16];
    const int k = blockIdx.y;
    const double *ak = alpha + (int64_t)k * m;
    const double *bk = beta + (int64_t)k * (m + 1);
    const bool live = first_break(ak, bk, j - 1) == 0;
    double a = sum_partials(dotpart + (int64_t)k * nblk, nblk, sh);
    if (!live) a = 0.0;
    int64_t beg, end;
    elem_range(n, nblk, beg, end);
    const int64_t base = (int64_t)k * n;
    double acc = 0.0;
    for (int64_t e = beg + threadIdx.x; e < end; e += blockDim.x) {
        double2 q = q_cur[base + e], v = w[base + e];
        v.x -= a * q.x;
        v.y -= a * q.y;
        w[base + e] = v;
        acc += v.x * v.x + v.y * v.y;
    }
    if (want_norm) {
        acc = block_sum(acc, sh);
        if (threadIdx.x == 0) nrmpart[(int64_t)k * nblk + blockIdx.x] = acc;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) alpha[(int64_t)k * m + (j - 1)] = a;
}

// Partial sums of h_i = <Q_i, w> for the nvec stored Lanczos vectors.
__global__ void __launch_bounds__(256) k_reorth_dots(const double2 *__restrict__ Q, int nvec,
                                                     int64_t slot, int64_t n, const double2 *__restrict__ w,
                                                     int nblk, double2 *__restrict__ hpart) {
    __shared__ double sh[16];
    const int k = blockIdx.y;
    int64_t beg, end;
    elem_range(n, nblk, beg, end);
    const int64_t base = (int64_t)k * n;
    for (int i = 0; i < nvec; ++i) {
        const double2 *qi = Q + i * slot + base;
        double re = 0.0, im = 0.0;
        for (int64_t e = beg + threadIdx.x; e < end; e += blockDim.x) {
            double2 q = qi[e], v = w[base + e];
            re += q.x * v.x + q.y * v.y;   // conj(q) * v
            im += q.x * v.y - q.y * v.x;
        }
        re = block_sum(re, sh);
        im = block_sum(im, sh);
        if (threadIdx.x == 0) hpart[((int64_t)k * nvec + i) * nblk + blockIdx.x] = make_double2(re, im);
    }
}

__global__ void k_reorth_reduce(const double2 *__restrict__ hpart, int nvec, int nblk,
                                double2 *__restrict__ h) {
    const int k = blockIdx.x;
    for (int i = threadIdx.x; i < nvec; i += blockDim.x) {
        const double2 *p = hpart + ((int64_t)k * nvec + i) * nblk;
        double re = 0.0, im = 0.0;
        for (int b = 0; b < nblk; ++b) {
            re += p[b].x;
            im += p[b].y;
        }
        h[(int64_t)k * nvec + i] = make_double2(re, im);
    }
}

// w -= sum_i h_i Q_i; optional partial sums of |w|^2.
__global__ void __launch_bounds__(256) k_reorth_update(const double2 *__restrict__ Q, int nvec, int64_t slot,
                                                       int64_t n, const double2 *__restrict__ h,
                                                       double2 *__restrict__ w, int nblk,
                                                       double *__restrict__ nrmpart, int want_norm) {
    __shared__ double sh[16];
    __shared__ double2 hs[TNSLQ_MAX_STEPS + 1];
    const int k = blockIdx.y;
    for (int i = threadIdx.x; i < nvec; i += blockDim.x) hs[i] = h[(int64_t)k * nvec + i];
    __syncthreads();
    int64_t beg, end;
    elem_range(n, nblk, beg, end);
    const int64_t base = (int64_t)k * n;
    double acc = 0.0;
    for (int64_t e = beg + threadIdx.x; e < end; e += blockDim.x) {
        double2 v = w[base + e];
        for (int i = 0; i < nvec; ++i) {
            double2 q = Q[i * slot + base + e], c = hs[i];
            v.x -= c.x * q.x - c.y * q.y;
            v.y -= c.x * q.y + c.y * q.x;
        }
        w[base + e] = v;
        acc += v.x * v.x + v.y * v.y;
    }
    if (want_norm) {
        acc = block_sum(acc, sh);
        if (threadIdx.x == 0) nrmpart[(int64_t)k * nblk + blockIdx.x] = acc;
    }
}

// beta_{j+1} = ||w||, breakdown test, q_{j+1} = w / beta_{j+1} (0 after a
// breakdown), and the transposed low-precision copy for the next contraction.
template <int PREC>
__global__ void __launch_bounds__(256) k_passC(const double *__restrict__ nrmpart, int64_t n, int64_t dA,
                                               int64_t dB, const double2 *__restrict__ w,
                                               double2 *__restrict__ q_next, void *__restrict__ Xt,
                                               int64_t xt_nst, const double *__restrict__ alpha,
                                               double *__restrict__ beta, int m, int j, int nblk) {
    __shared__ double sh[16];
    const int k = blockIdx.y;
    const double *ak = alpha + (int64_t)k * m;
    double *bk = beta + (int64_t)k * (m + 1);
    const bool live = first_break(ak, bk, j - 1) == 0;
    double b = sqrt(sum_partials(nrmpart + (int64_t)k * nblk, nblk, sh));
    if (!live) b = 0.0;
    bool cont = live;
    if (live) {
        double amax = 0.0, bmax = 0.0;
        for (int s = 1; s <= j; ++s) {
            amax = fmax(amax, fabs(ak[s - 1]));
            if (s >= 2) bmax = fmax(bmax, bk[s - 1]);
        }
        if (b <= BREAKDOWN_TOL * (amax + bmax)) cont = false;
    }
    const int64_t base = (int64_t)k * n;
    const int64_t gstride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gstride) {
        double2 v = w[base + e];
        double2 q = cont ? make_double2(v.x / b, v.y / b) : make_double2(0.0, 0.0);
        q_next[base + e] = q;
        // Xt entry (row (k, b'), reduction index a') reads w at a' * dB + b'
        if (Xt) {
            const int64_t bb = e / dA, aa = e % dA;
            double2 u = w[base + aa * dB + bb];
            double2 qt = cont ? make_double2(u.x / b, u.y / b) : make_double2(0.0, 0.0);
            store_planes<PREC>(Xt, brick_ps(PREC), brick_index(PREC, xt_nst, (int64_t)k * dB + bb, aa), qt.x,
                               qt.y);
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) bk[j] = b;
}

__global__ void k_steps(const double *__restrict__ alpha, const double *__restrict__ beta, int K, int m,
                        int jdone, int *__restrict__ steps) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= K) return;
    const int s = first_break(alpha + (int64_t)k * m, beta + (int64_t)k * (m + 1), jdone);
    steps[k] = s ? s : jdone;
}

// Eigenvalues and first eigenvector components of the symmetric tridiagonal
// (d, e) by implicit QL with Wilkinson-type shifts (Bowdler, Martin, Reinsch
// & Wilkinson 1968), accumulating only the first row of the eigenvector
// matrix.  e[i] couples d[i] and d[i+1]; e[n-1] must be 0.  On return d holds
// the eigenvalues and z the first components.  Entry i of each array sits at
// index i * ST (the arrays of several threads interleaved in LDS).
template <int ST>
__device__ void tridiag_ql_first_row(int n, double *d_, double *e_, double *z_) {
    auto d = [&](int i) -> double & { return d_[i * ST]; };
    auto e = [&](int i) -> double & { return e_[i * ST]; };
    auto z = [&](int i) -> double & { return z_[i * ST]; };
    for (int i = 0; i < n; ++i) z(i) = (i == 0) ? 1.0 : 0.0;
    for (int l = 0; l < n; ++l) {
        int iter = 0;
        while (true) {
            int mm = l;
            for (; mm < n - 1; ++mm) {
                const double dd = fabs(d(mm)) + fabs(d(mm + 1));
                if (fabs(e(mm)) <= DBL_EPSILON * dd) break;
            }
            if (mm == l || ++iter > 64) break;
            double g = (d(l + 1) - d(l)) / (2.0 * e(l));
            double r = hypot(g, 1.0);
            g = d(mm) - d(l) + e(l) / (g + copysign(r, g));
            double s = 1.0, c = 1.0, p = 0.0;
            bool early = false;
            for (int i = mm - 1; i >= l; --i) {
                const double f = s * e(i), bb = c * e(i);
                r = hypot(f, g);
                e(i + 1) = r;
                if (r == 0.0) {
                    d(i + 1) -= p;
                    e(mm) = 0.0;
                    early = true;
                    break;
                }
                s = f / r;
                c = g / r;
                g = d(i + 1) - p;
                r = (d(i) - g) * s + 2.0 * c * bb;
                p = s * r;
                d(i + 1) = g + p;
                g = c * r - bb;
                const double fz = z(i + 1);
                z(i + 1) = s * z(i) + c * fz;
                z(i) = c * z(i) - s * fz;
            }
            if (early) continue;
            d(l) -= p;
            e(l) = g;
            e(mm) = 0.0;
        }
    }
}

// F[k][j-1] = sum_i tau_i^2 |theta_i| for T_j (j capped at steps[k]).
// f of the quadrature: TNSLQ_F_ABS |x| (the negativity), TNSLQ_F_ENTROPY
// -x log2 x (0 for x <= 0), TNSLQ_F_PURITY x^2.
__device__ inline double quad_f(int fn, double x) {
    if (fn == TNSLQ_F_ENTROPY) return x > 0.0 ? -x * log2(x) : 0.0;
    if (fn == TNSLQ_F_PURITY) return x * x;
    return fabs(x);
}

// One thread per (probe, step); the threads of a block keep their d, e, z in
// LDS, entry i of thread t at [i][t] (consecutive threads, consecutive banks).
constexpr int QD_THREADS = 32;
__global__ void __launch_bounds__(QD_THREADS) k_quadrature(const double *__restrict__ alpha,
                                                           const double *__restrict__ beta,
                                                           const int *__restrict__ steps, int K, int m, int jlo,
                                                           int jhi, int fn, double *__restrict__ F) {
    __shared__ double sd[TNSLQ_MAX_STEPS * QD_THREADS], se[TNSLQ_MAX_STEPS * QD_THREADS],
        sz[TNSLQ_MAX_STEPS * QD_THREADS];
    const int nj = jhi - jlo + 1;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= K * nj) return;
    const int k = t / nj, j = jlo + t % nj;
    int jj = j;
    if (steps && steps[k] < jj) jj = steps[k];
    double *d = sd + threadIdx.x, *e = se + threadIdx.x, *z = sz + threadIdx.x;
    for (int i = 0; i < jj; ++i) {
        d[i * QD_THREADS] = alpha[(int64_t)k * m + i];
        e[i * QD_THREADS] = (i + 1 < jj) ? beta[(int64_t)k * (m + 1) + i + 1] : 0.0;
    }
    tridiag_ql_first_row<QD_THREADS>(jj, d, e, z);
    double f = 0.0;
    for (int i = 0; i < jj; ++i) {
        const double zi = z[i * QD_THREADS];
        f += zi * zi * quad_f(fn, d[i * QD_THREADS]);
    }
    F[(int64_t)k * m + (j - 1)] = f;
}

// G_k = beta_1^2 F_j; mean, SE = sqrt(Var / K) (sample variance), E = log2 mean,
// dE = SE / (mean ln 2).  stats[(j-1)*4 + {0,1,2,3}].
__global__ void __launch_bounds__(256) k_stats(const double *__restrict__ beta, const double *__restrict__ F,
                                               int K, int m, int j, double *__restrict__ G,
                                               double *__restrict__ stats) {
    __shared__ double sh[16];
    double s = 0.0;
    for (int k = threadIdx.x; k < K; k += blockDim.x) {
        const double b1 = beta[(int64_t)k * (m + 1)];
        const double g = b1 * b1 * F[(int64_t)k * m + (j - 1)];
        if (G) G[k] = g;
        s += g;
    }
    const double mean = block_sum(s, sh) / K;
    double v = 0.0;
    for (int k = threadIdx.x; k < K; k += blockDim.x) {
        const double b1 = beta[(int64_t)k * (m + 1)];
        const double g = b1 * b1 * F[(int64_t)k * m + (j - 1)];
        v += (g - mean) * (g - mean);
    }
    v = block_sum(v, sh);
    if (threadIdx.x == 0) {
        const double nan = __longlong_as_double(0x7ff8000000000000ll);
        const double se = K > 1 ? sqrt(v / (K - 1) / K) : nan;
        double *o = stats + (int64_t)(j - 1) * 4;
        o[0] = mean;
        o[1] = se;
        o[2] = log2(mean);
        o[3] = K > 1 ? se / (mean * 0.69314718055994530942) : nan;
    }
}

// ---------------------------------------------------------------- fit
// lanczos_estimate of Sec. III: a least-squares fit of F_inf + a r^t to the
// last FIT_WINDOW quadrature values of a probe, leaving out F_1 (the one-node
// rule) (t = 0 at the first point of the window), r in [-FIT_R_MAX, FIT_R_MAX] so that the sign-alternating approach
// of the |x| quadrature is an exponential too.  For fixed r the fit is the
// linear regression of the values on r^t; r is chosen on an even grid of
// FIT_GRID points and refined by golden-section search between the best grid
// point's neighbours.  The fit's own uncertainty of F_inf is sqrt(C_00) of
// C = RSS / (n - 3) (J^T J)^-1, J the model's Jacobian in (F_inf, a, r); an
// exact fit has uncertainty 0, a singular J^T J with RSS > 0 infinity.  To it
// is added in quadrature the model error: the distance from F_inf to the limit
// F_alg of the algebraic law F_j = F_alg + c (-1)^j / j^2 + d / j^2 (j the step
// number) fitted to the same window by linear least squares, the way Gauss
// quadrature of a function with a kink approaches its limit.  A probe whose
// recurrence broke down by step j is exact: F_s, uncertainty 0.
constexpr int FIT_WINDOW = TNSLQ_FIT_WINDOW;
constexpr int FIT_MIN_POINTS = TNSLQ_FIT_MIN_POINTS;
constexpr int FIT_GRID = 397;
constexpr double FIT_R_MAX = 0.99;

// RSS of the regression y_t ~ f + a r^t (t = 0..n-1), with f, a.
__device__ inline double fit_linear(const double *y, int n, double r, double &f, double &a) {
    double x[FIT_WINDOW];
    double p = 1.0, mx = 0.0, my = 0.0;
    for (int t = 0; t < n; ++t) {
        x[t] = p;
        p *= r;
        mx += x[t];
        my += y[t];
    }
    mx /= n;
    my /= n;
    double sxx = 0.0, sxy = 0.0;
    for (int t = 0; t < n; ++t) {
        sxx += (x[t] - mx) * (x[t] - mx);
        sxy += (x[t] - mx) * (y[t] - my);
    }
    a = sxx > 0.0 ? sxy / sxx : 0.0;
    f = my - a * mx;
    double rss = 0.0;
    for (int t = 0; t < n; ++t) {
        const double e = y[t] - f - a * x[t];
        rss += e * e;
    }
    return rss;
}

__device__ inline double fit_grid_r(int i) { return -FIT_R_MAX + (2.0 * FIT_R_MAX) * i / (FIT_GRID - 1); }

// F_alg of the least-squares fit of F_alg + c (-1)^j / j^2 + d / j^2 to the n
// values y of steps j0 .. j0 + n - 1: the two decaying columns are
// orthonormalised (Gram-Schmidt, each projection applied twice) and F_alg is
// the regression of y on the constant column's remainder.
__device__ inline double fit_algebraic(const double *y, int n, int j0) {
    double q[2][FIT_WINDOW], one[FIT_WINDOW], yr[FIT_WINDOW];
    for (int t = 0; t < n; ++t) {
        const double jj = (double)(j0 + t), w = 1.0 / (jj * jj);
        q[0][t] = ((j0 + t) & 1) ? -w : w;
        q[1][t] = w;
        one[t] = 1.0;
        yr[t] = y[t];
    }
    auto dot = [&](const double *u, const double *v) {
        double s = 0.0;
        for (int t = 0; t < n; ++t) s += u[t] * v[t];
        return s;
    };
    auto remove = [&](double *v, const double *u) {
        for (int pass = 0; pass < 2; ++pass) {
            const double c = dot(u, v);
            for (int t = 0; t < n; ++t) v[t] -= c * u[t];
        }
    };
    for (int c = 0; c < 2; ++c) {
        if (c == 1) remove(q[1], q[0]);
        const double nr = sqrt(dot(q[c], q[c]));
        for (int t = 0; t < n; ++t) q[c][t] /= nr;
    }
    for (int c = 0; c < 2; ++c) {
        remove(one, q[c]);
        remove(yr, q[c]);
    }
    return dot(one, yr) / dot(one, one);
}

// Per probe k (one wave each): F_inf and its uncertainty after step
// j >= FIT_MIN_POINTS + 1.  The lanes share the grid; the first grid point of
// least RSS wins (as a scan in order would pick it), and lane 0 refines it.
__global__ void __launch_bounds__(64) k_fit(const double *__restrict__ alpha, const double *__restrict__ beta,
                                            const double *__restrict__ F, int K, int m, int j,
                                            double *__restrict__ finf, double *__restrict__ fsig) {
    const int k = blockIdx.x, lane = threadIdx.x;
    if (k >= K) return;
    const double *ak = alpha + (int64_t)k * m, *bk = beta + (int64_t)k * (m + 1), *Fk = F + (int64_t)k * m;
    const int s = first_break(ak, bk, j);
    if (s > 0) {
        if (lane == 0) {
            finf[k] = Fk[s - 1];
            fsig[k] = 0.0;
        }
        return;
    }
    const int lo = j - FIT_WINDOW > 1 ? j - FIT_WINDOW : 1;   // F_1 is never fitted
    const int n = j - lo;
    double y[FIT_WINDOW];
    for (int t = 0; t < n; ++t) y[t] = Fk[lo + t];
    double f, a, best = INFINITY;
    int ib = FIT_GRID;   // none yet
    for (int i = lane; i < FIT_GRID; i += 64) {
        const double rss = fit_linear(y, n, fit_grid_r(i), f, a);
        if (rss < best) {
            best = rss;
            ib = i;
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        const double ob = __shfl_xor(best, off, 64);
        const int oi = __shfl_xor(ib, off, 64);
        if (ob < best || (ob == best && oi < ib)) {
            best = ob;
            ib = oi;
        }
    }
    if (lane != 0) return;
    if (ib == FIT_GRID) ib = 0;
    double lo_r = fit_grid_r(ib > 0 ? ib - 1 : 0), hi_r = fit_grid_r(ib < FIT_GRID - 1 ? ib + 1 : FIT_GRID - 1);
    const double g = 0.61803398874989484820;   // (sqrt(5) - 1) / 2
    double x1 = hi_r - g * (hi_r - lo_r), x2 = lo_r + g * (hi_r - lo_r);
    double f1 = fit_linear(y, n, x1, f, a), f2 = fit_linear(y, n, x2, f, a);
    for (int it = 0; it < 200 && hi_r - lo_r > 1e-13; ++it) {
        if (f1 <= f2) {
            hi_r = x2;
            x2 = x1;
            f2 = f1;
            x1 = hi_r - g * (hi_r - lo_r);
            f1 = fit_linear(y, n, x1, f, a);
        } else {
            lo_r = x1;
            x1 = x2;
            f1 = f2;
            x2 = lo_r + g * (hi_r - lo_r);
            f2 = fit_linear(y, n, x2, f, a);
        }
    }
    double r = 0.5 * (lo_r + hi_r);
    double rss = fit_linear(y, n, r, f, a);
    if (!(rss <= best)) {
        r = fit_grid_r(ib);
        rss = fit_linear(y, n, r, f, a);
    }
    double sig;
    if (rss == 0.0) {
        sig = 0.0;
    } else {
        // J^T J for the columns 1, r^t, a t r^(t-1)
        double m00 = 0, m01 = 0, m02 = 0, m11 = 0, m12 = 0, m22 = 0;
        double p = 1.0, pm = 1.0;   // r^t, r^(t-1) (taken as 1 at t = 0, where the column is 0)
        for (int t = 0; t < n; ++t) {
            const double c1 = p, c2 = t > 0 ? a * t * pm : 0.0;
            m00 += 1.0;
            m01 += c1;
            m02 += c2;
            m11 += c1 * c1;
            m12 += c1 * c2;
            m22 += c2 * c2;
            pm = p;
            p *= r;
        }
        const double cof00 = m11 * m22 - m12 * m12;
        const double det = m00 * cof00 - m01 * (m01 * m22 - m12 * m02) + m02 * (m01 * m12 - m11 * m02);
        const double c00 = rss / (n - 3) * cof00 / det;
        sig = (det > 0.0 && isfinite(c00) && c00 >= 0.0) ? sqrt(c00) : INFINITY;
    }
    const double dm = f - fit_algebraic(y, n, lo + 1);
    finf[k] = f;
    fsig[k] = isfinite(sig) ? sqrt(sig * sig + dm * dm) : sig;
}

// Block statistics of the fitted estimates: G_n = beta_1^2 F_inf,n;
// out = {mean T, SE (N - 1), eps_L = mean beta_1^2 sigma_n, E = log2 T,
//        dE = sqrt(SE^2 + eps_L^2) / (T ln 2), SE / (T ln 2)}.
__global__ void __launch_bounds__(256) k_fit_stats(const double *__restrict__ beta, const double *__restrict__ finf,
                                                   const double *__restrict__ fsig, int K, int m,
                                                   double *__restrict__ G, double *__restrict__ out) {
    __shared__ double sh[16];
    double s = 0.0, e = 0.0;
    for (int k = threadIdx.x; k < K; k += blockDim.x) {
        const double b1 = beta[(int64_t)k * (m + 1)];
        const double g = b1 * b1 * finf[k];
        if (G) G[k] = g;
        s += g;
        e += b1 * b1 * fsig[k];
    }
    const double mean = block_sum(s, sh) / K;
    const double eps = block_sum(e, sh) / K;
    double v = 0.0;
    for (int k = threadIdx.x; k < K; k += blockDim.x) {
        const double b1 = beta[(int64_t)k * (m + 1)];
        const double g = b1 * b1 * finf[k];
        v += (g - mean) * (g - mean);
    }
    v = block_sum(v, sh);
    if (threadIdx.x == 0) {
        const double ln2 = 0.69314718055994530942;
        const double se = K > 1 ? sqrt(v / (K - 1) / K) : 0.0;
        out[0] = mean;
        out[1] = se;
        out[2] = eps;
        out[3] = log2(mean);
        out[4] = sqrt(se * se + eps * eps) / (mean * ln2);
        out[5] = K > 1 ? se / (mean * ln2) : __longlong_as_double(0x7ff8000000000000ll);
    }
}

// Surrogate inputs: probe means of dAB alpha_1..n_early in slots 0..7 and of
// dAB beta_2..n_early+1 in slots 8..15 (slots past n_early hold zero), then
// log2 dA, log2 dB, log2 dE.
__global__ void k_features(const double *__restrict__ alpha, const double *__restrict__ beta, int K, int m,
                           int n_early, double dAB, double dA, double dB, double dE, float *__restrict__ feat) {
    const int t = threadIdx.x;
    if (t < 2 * TNSLQ_SURROGATE_MAX_EARLY) {
        const bool is_a = t < TNSLQ_SURROGATE_MAX_EARLY;
        const int i = is_a ? t : t - TNSLQ_SURROGATE_MAX_EARLY;
        double s = 0.0;
        if (i < n_early)
            for (int k = 0; k < K; ++k)
                s += is_a ? alpha[(int64_t)k * m + i] : beta[(int64_t)k * (m + 1) + i + 1];
        feat[t] = (float)(dAB * s / K);
    } else if (t < 2 * TNSLQ_SURROGATE_MAX_EARLY + 3) {
        const int i = t - 2 * TNSLQ_SURROGATE_MAX_EARLY;
        feat[t] = (float)log2(i == 0 ? dA : (i == 1 ? dB : dE));
    }
}

inline unsigned cdiv(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

}  // namespace

hipError_t launch_passA(int accfp64, const LzDims &z, const void *part, int S, int64_t split_stride, int k0,
                        int kc, const double2 *q_prev, const double2 *q_cur, double2 *w, const double *alpha,
                        const double *beta, int j, double *dotpart, hipStream_t st) {
    dim3 grid(z.nblk, kc), block(256);
    if (accfp64)
        hipLaunchKernelGGL((k_passA<double2>), grid, block, 0, st, (const double2 *)part, S, split_stride, k0,
                           z.n, q_prev, q_cur, w, alpha, beta, z.m, j, z.nblk, dotpart);
    else
        hipLaunchKernelGGL((k_passA<float2>), grid, block, 0, st, (const float2 *)part, S, split_stride, k0,
                           z.n, q_prev, q_cur, w, alpha, beta, z.m, j, z.nblk, dotpart);
    return hipGetLastError();
}

hipError_t launch_passB(const LzDims &z, const double *dotpart, const double2 *q_cur, double2 *w,
                        double *alpha, const double *beta, int j, double *nrmpart, int want_norm,
                        hipStream_t st) {
    dim3 grid(z.nblk, z.K), block(256);
    hipLaunchKernelGGL(k_passB, grid, block, 0, st, dotpart, z.n, q_cur, w, alpha, beta, z.m, j, z.nblk,
                       nrmpart, want_norm);
    return hipGetLastError();
}

hipError_t launch_reorth(const LzDims &z, const double2 *Q, int nvec, int64_t slot, double2 *w,
                         double *hpart, double2 *h, const double *alpha, const double *beta, int j,
                         double *nrmpart, hipStream_t st) {
    (void)alpha;
    (void)beta;
    (void)j;
    dim3 grid(z.nblk, z.K), block(256);
    for (int pass = 0; pass < 2; ++pass) {
        hipLaunchKernelGGL(k_reorth_dots, grid, block, 0, st, Q, nvec, slot, z.n, (const double2 *)w, z.nblk,
                           (double2 *)hpart);
        hipLaunchKernelGGL(k_reorth_reduce, dim3(z.K), dim3(64), 0, st, (const double2 *)hpart, nvec, z.nblk, h);
        hipLaunchKernelGGL(k_reorth_update, grid, block, 0, st, Q, nvec, slot, z.n, (const double2 *)h, w,
                           z.nblk, nrmpart, pass == 1 ? 1 : 0);
    }
    return hipGetLastError();
}

hipError_t launch_passC(int prec, const LzDims &z, const double *nrmpart, const double2 *w, double2 *q_next,
                        void *Xt, int64_t xt_nst, const double *alpha, double *beta, int j, hipStream_t st) {
    dim3 grid(z.nblk, z.K), block(256);
#define TNSLQ_PC(P)                                                                                         \
    hipLaunchKernelGGL((k_passC<P>), grid, block, 0, st, nrmpart, z.n, z.dA, z.dB, w, q_next, Xt, xt_nst, \
                       alpha, beta, z.m, j, z.nblk)
    switch (prec) {
        case TNSLQ_FP64: TNSLQ_PC(TNSLQ_FP64); break;
        case TNSLQ_FP32: TNSLQ_PC(TNSLQ_FP32); break;
        case TNSLQ_BF16X3: TNSLQ_PC(TNSLQ_BF16X3); break;
        default: TNSLQ_PC(TNSLQ_BF16X6); break;
    }
#undef TNSLQ_PC
    return hipGetLastError();
}

hipError_t launch_steps(const double *alpha, const double *beta, int K, int m, int jdone, int *steps,
                        hipStream_t st) {
    hipLaunchKernelGGL(k_steps, dim3(cdiv(K, 64)), dim3(64), 0, st, alpha, beta, K, m, jdone, steps);
    return hipGetLastError();
}

hipError_t launch_quadrature(const double *alpha, const double *beta, const int *steps, int K, int m, int jlo,
                             int jhi, int fn, double *F, hipStream_t st) {
    const int64_t nt = (int64_t)K * (jhi - jlo + 1);
    hipLaunchKernelGGL(k_quadrature, dim3(cdiv(nt, QD_THREADS)), dim3(QD_THREADS), 0, st, alpha, beta, steps, K, m, jlo, jhi, fn, F);
    return hipGetLastError();
}

hipError_t launch_stats(const double *beta, const double *F, int K, int m, int j, double *G, double *stats,
                        hipStream_t st) {
    hipLaunchKernelGGL(k_stats, dim3(1), dim3(256), 0, st, beta, F, K, m, j, G, stats);
    return hipGetLastError();
}

hipError_t launch_fit(const double *alpha, const double *beta, const double *F, int K, int m, int j, double *finf,
                      double *fsig, double *G, double *out, hipStream_t st) {
    if (j < FIT_MIN_POINTS + 1 || j > m) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_fit, dim3(K), dim3(64), 0, st, alpha, beta, F, K, m, j, finf, fsig);
    hipLaunchKernelGGL(k_fit_stats, dim3(1), dim3(256), 0, st, beta, (const double *)finf, (const double *)fsig, K, m,
                       G, out);
    return hipGetLastError();
}

hipError_t launch_features(const double *alpha, const double *beta, int K, int m, int n_early, double dAB,
                           double dA, double dB, double dE, float *feat, hipStream_t st) {
    hipLaunchKernelGGL(k_features, dim3(1), dim3(64), 0, st, alpha, beta, K, m, n_early, dAB, dA, dB, dE, feat);
    return hipGetLastError();
}

}  // namespace tnslq
