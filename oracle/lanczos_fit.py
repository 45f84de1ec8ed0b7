"""Adaptive stopping of stochastic Lanczos quadrature: the exponential fit
behind Algorithm 1's lanczos_converged / lanczos_estimate (Sec. III), and the
error on the Hutchinson mean behind hutchinson_converged.

Oracle, test infrastructure only.

Sec. III proposes a least-squares fit of an exponential to the quadrature
values F_1..F_k of one probe: the fit's equilibrium value estimates the
bilinear form and its uncertainty is the error tested for convergence.  The
paper fixes neither the points, the weights nor the form of the exponential;
the readings taken here (each also listed in the design notes):

  * model F_t = F_inf + a r^t over the last FIT_WINDOW quadrature values
    (fewer early on), t = 0, 1, ... counted from the first point of the window,
    unweighted.  F_1, the one-node rule (|alpha_1|, far from every later
    value), is never fitted, so the window holds F_max(2, k-FIT_WINDOW+1)..F_k;  The ratio r = +-exp(-b) ranges over
    [-FIT_R_MAX, FIT_R_MAX]: for |x| the quadrature values of successive
    Lanczos steps fall on alternate sides of the limit, an exponential approach
    with sign-alternating ratio;
  * at least FIT_MIN_POINTS points (two degrees of freedom for the residual),
    so the first fit comes after step FIT_MIN_POINTS + 1;
  * uncertainty of F_inf = sqrt(C_00) of the linearised covariance
    C = s^2 (J^T J)^-1, s^2 = RSS / (n - 3), J the Jacobian of the model in
    (F_inf, a, r) at the optimum; an exact fit (RSS = 0) has uncertainty 0, a
    fit with singular J^T J and RSS > 0 has uncertainty inf;
  * the exponential is a model, and the covariance measures only how well it
    fits the window, not how the quadrature of |x| really approaches its
    limit.  That approach is algebraic: Gauss quadrature of a function with a
    kink converges like 1/j^2 in the number of nodes j, on alternate sides.
    So the same window is also fitted, by linear least squares, with
    F_j = F_alg + c (-1)^j / j^2 + d / j^2 (j the step number), and the
    difference between the two extrapolations is added in quadrature:
    sigma = sqrt(C_00 + (F_inf - F_alg)^2).  The estimate stays the
    exponential fit's F_inf.  Without this term the stated error covered the
    error against long runs on 42% of a set of Haar states (the exponential
    extrapolation falls short of the limit on every one of them);
  * a probe whose Lanczos recurrence broke down at step s <= k is exact:
    estimate F_s, uncertainty 0;
  * a run with a target that no step up to the last one meets reports the
    plain quadrature estimate of its last step (Algorithm 1's estimate
    without the extrapolation), with the fit's Lanczos error at that step:
    the fitted limit of a trajectory that has not settled can be several bits
    off where the plain estimate is not (brickwork states with many small
    eigenvalues of rho^{T_B}).

Fitting method (the definition is the least-squares optimum; this is how it
is found): for fixed r the model is linear in (F_inf, a) and solved by linear
least squares; the residual sum of squares is scanned over FIT_GRID evenly
spaced r in [-FIT_R_MAX, FIT_R_MAX] and the best grid point refined by bounded
scalar minimisation between its neighbours.
"""
from __future__ import annotations

from typing import Dict

import numpy as np
import scipy.optimize

from . import step_difference
from .slq import BREAKDOWN_TOL

FIT_WINDOW = 8
FIT_MIN_POINTS = 5
FIT_R_MAX = 0.99
FIT_GRID = 397


def _linear_part(y: np.ndarray, r: float):
    """(F_inf, a) minimising sum_t (y_t - F_inf - a r^t)^2, and the RSS."""
    t = np.arange(y.size, dtype=np.float64)
    B = np.stack([np.ones_like(t), r ** t], axis=1)
    coef, *_ = np.linalg.lstsq(B, y, rcond=None)
    res = y - B @ coef
    return float(coef[0]), float(coef[1]), float(res @ res)


def exponential_fit(y) -> Dict[str, float]:
    """Least-squares fit of F_inf + a r^t (t = 0..n-1) to the values y.

    Returns F_inf, a, r, rss and sigma (the uncertainty of F_inf)."""
    y = np.asarray(y, dtype=np.float64)
    n = y.size
    if n < FIT_MIN_POINTS:
        raise ValueError(f"need at least {FIT_MIN_POINTS} points, got {n}")
    grid = np.linspace(-FIT_R_MAX, FIT_R_MAX, FIT_GRID)
    rss = np.array([_linear_part(y, r)[2] for r in grid])
    i = int(np.argmin(rss))
    lo, hi = grid[max(i - 1, 0)], grid[min(i + 1, FIT_GRID - 1)]
    opt = scipy.optimize.minimize_scalar(lambda r: _linear_part(y, r)[2], bounds=(lo, hi), method="bounded",
                                         options={"xatol": 1e-13})
    r = float(opt.x) if opt.fun <= rss[i] else float(grid[i])
    f_inf, a, rss_opt = _linear_part(y, r)
    if rss_opt == 0.0:
        sigma = 0.0
    else:
        t = np.arange(n, dtype=np.float64)
        dr = np.where(t > 0, a * t * r ** np.maximum(t - 1, 0), 0.0)
        J = np.stack([np.ones(n), r ** t, dr], axis=1)
        JtJ = J.T @ J
        try:
            C = (rss_opt / (n - 3)) * np.linalg.inv(JtJ)
            sigma = float(np.sqrt(C[0, 0])) if np.isfinite(C[0, 0]) and C[0, 0] >= 0 else float("inf")
        except np.linalg.LinAlgError:
            sigma = float("inf")
    return {"f_inf": f_inf, "a": a, "r": r, "rss": rss_opt, "sigma": sigma}


def algebraic_fit(y, j_end: int) -> float:
    """F_alg of the least-squares fit of F_alg + c (-1)^j / j^2 + d / j^2 to
    the values y of steps j = j_end - len(y) + 1 .. j_end."""
    y = np.asarray(y, dtype=np.float64)
    n = y.size
    if n < 3:
        raise ValueError("the algebraic model has three parameters")
    j = np.arange(j_end - n + 1, j_end + 1, dtype=np.float64)
    B = np.stack([np.ones(n), (-1.0) ** j / (j * j), 1.0 / (j * j)], axis=1)
    coef, *_ = np.linalg.lstsq(B, y, rcond=None)
    return float(coef[0])


def breakdown_step(alpha, beta) -> int:
    """Step s at which the recurrence broke down (beta_{s+1} <= 1e-12 (max_i<=s
    |alpha_i| + max_2<=i<=s beta_i), the rule of the Lanczos oracle), or 0."""
    amax = bmax = 0.0
    for s in range(1, len(alpha) + 1):
        amax = max(amax, abs(alpha[s - 1]))
        if s >= 2:
            bmax = max(bmax, beta[s - 1])
        if beta[s] <= BREAKDOWN_TOL * (amax + bmax):
            return s
    return 0


def lanczos_estimate(F_traj, k: int, broke: int = 0) -> Dict[str, float]:
    """lanczos_estimate and its uncertainty for one probe after k Lanczos
    steps, from its quadrature values F_traj[0..k-1] (F_traj[j-1] = F_j);
    `broke` is the step of a breakdown, 0 if none.  sigma combines the fit's
    own uncertainty (sigma_fit) and the model term (model)."""
    F_traj = np.asarray(F_traj, dtype=np.float64)
    if 0 < broke <= k:
        return {"f_inf": float(F_traj[broke - 1]), "sigma": 0.0, "sigma_fit": 0.0, "model": 0.0}
    lo = max(1, k - FIT_WINDOW)
    fit = exponential_fit(F_traj[lo:k])
    model = abs(fit["f_inf"] - algebraic_fit(F_traj[lo:k], k))
    return {"f_inf": fit["f_inf"], "sigma": float(np.hypot(fit["sigma"], model)), "sigma_fit": fit["sigma"],
            "model": model}


def fit_stats(F: np.ndarray, alpha: np.ndarray, beta: np.ndarray, k: int) -> Dict[str, float]:
    """Block estimate after k steps with every probe's fit: G_n = beta_1^2
    F_inf,n; mean T, Hutchinson error SE (sample variance, N - 1), Lanczos
    error eps_L = mean_n beta_1^2 sigma_n (the probes' fit errors are taken as
    fully correlated), E = log2 T and the combined error of E,
    dE = sqrt(SE^2 + eps_L^2) / (T ln 2)."""
    K = F.shape[0]
    G = np.zeros(K)
    S = np.zeros(K)
    for n in range(K):
        est = lanczos_estimate(F[n], k, breakdown_step(alpha[n], beta[n]))
        G[n] = beta[n, 0] ** 2 * est["f_inf"]
        S[n] = beta[n, 0] ** 2 * est["sigma"]
    T = float(np.mean(G))
    se = float(np.std(G, ddof=1) / np.sqrt(K)) if K > 1 else 0.0
    eps_l = float(np.mean(S))
    e = float(np.log2(T))
    de = float(np.sqrt(se * se + eps_l * eps_l) / (T * np.log(2.0)))
    return {"G": G, "sigma": S, "trace_norm": T, "trace_norm_se": se, "lanczos_err": eps_l, "logneg": e,
            "logneg_err": de}


def fit_stop_step(F: np.ndarray, alpha: np.ndarray, beta: np.ndarray, tol: float) -> int:
    """First step k >= FIT_MIN_POINTS + 1 whose combined error meets
    dE <= tol max(|E|, 1) (the +-tol target in bits, relative), else the last
    step."""
    m = F.shape[1]
    for k in range(FIT_MIN_POINTS + 1, m + 1):
        s = fit_stats(F, alpha, beta, k)
        if np.isfinite(s["logneg_err"]) and s["logneg_err"] <= tol * max(abs(s["logneg"]), 1.0):
            return k
    return m


def fit_rule_result(F: np.ndarray, alpha: np.ndarray, beta: np.ndarray, tol: float) -> Dict[str, object]:
    """What a run under the fit rule with target tol > 0 reports: the fitted
    block estimate at the first step meeting the target, else the plain
    estimate of the last step with the fit's Lanczos error there (in bits)."""
    m = F.shape[1]
    k = fit_stop_step(F, alpha, beta, tol)
    st = fit_stats(F, alpha, beta, k)
    lanczos_bits = st["lanczos_err"] / (st["trace_norm"] * np.log(2.0))
    if np.isfinite(st["logneg_err"]) and st["logneg_err"] <= tol * max(abs(st["logneg"]), 1.0):
        return {"step": k, "met": True, "logneg": st["logneg"], "trace_norm": st["trace_norm"],
                "trace_norm_se": st["trace_norm_se"], "G": st["G"], "lanczos_err": lanczos_bits}
    plain = step_difference.block_estimate(beta, F, m)
    return {"step": m, "met": False, "logneg": plain["logneg"], "trace_norm": plain["trace_norm"],
            "trace_norm_se": plain["trace_norm_se"], "G": np.asarray(beta)[:, 0] ** 2 * np.asarray(F)[:, m - 1],
            "lanczos_err": lanczos_bits}


def block_lanczos_stop_step(F: np.ndarray, alpha: np.ndarray, beta: np.ndarray, tol: float) -> int:
    """lanczos_converged for a block of probes: the first step k >=
    FIT_MIN_POINTS + 1 whose Lanczos error alone meets the target,
    eps_L / (T ln 2) <= tol max(|E|, 1), else the last step."""
    m = F.shape[1]
    for k in range(FIT_MIN_POINTS + 1, m + 1):
        s = fit_stats(F, alpha, beta, k)
        lerr = s["lanczos_err"] / (s["trace_norm"] * np.log(2.0))
        if np.isfinite(lerr) and lerr <= tol * max(abs(s["logneg"]), 1.0):
            return k
    return m


def combined_stats(G: np.ndarray, S: np.ndarray) -> Dict[str, float]:
    """Estimate over all probes so far from their fitted G_n and Lanczos
    errors S_n = beta_1^2 sigma_n: T = mean G, SE (N - 1 variance),
    eps_L = mean S, E = log2 T, dE = sqrt(SE^2 + eps_L^2) / (T ln 2); with a
    single probe the Hutchinson error is unknown and dE is infinite."""
    G = np.asarray(G, dtype=np.float64)
    S = np.asarray(S, dtype=np.float64)
    N = G.size
    T = float(np.mean(G))
    se = float(np.std(G, ddof=1) / np.sqrt(N)) if N > 1 else float("nan")
    eps_l = float(np.mean(S))
    de = float(np.sqrt(se * se + eps_l * eps_l) / (T * np.log(2.0))) if N > 1 else float("inf")
    return {"trace_norm": T, "trace_norm_se": se, "lanczos_err": eps_l, "logneg": float(np.log2(T)),
            "logneg_err": de}


def probe_loop(block, n_probes: int, max_probes: int, tol: float) -> Dict[str, object]:
    """Algorithm 1's outer loop over probes, in blocks of n_probes: block b
    (block(b) -> its quadrature trajectories F, alpha, beta, with probe
    offsets b n_probes) runs until its own Lanczos error meets the target
    (block_lanczos_stop_step); its fitted G_n and S_n = beta_1^2 sigma_n join
    the earlier blocks'.  Blocks are added until the estimate over all probes
    meets dE <= tol max(|E|, 1) (hutchinson_converged) or the next block would
    pass max_probes."""
    G, S, stops = [], [], []
    b = 0
    while True:
        F, alpha, beta = block(b)
        k = block_lanczos_stop_step(F, alpha, beta, tol)
        st = fit_stats(F, alpha, beta, k)
        G.extend(st["G"])
        S.extend(st["sigma"])
        stops.append(k)
        c = combined_stats(np.array(G), np.array(S))
        if np.isfinite(c["logneg_err"]) and c["logneg_err"] <= tol * max(abs(c["logneg"]), 1.0):
            break
        if (b + 2) * n_probes > max_probes:
            break
        b += 1
    c.update({"G": np.array(G), "S": np.array(S), "stops": stops, "n_probes_used": len(G)})
    return c
