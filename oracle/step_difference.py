"""The step-difference stopping rule: a reading of Algorithm 1's
lanczos_converged / hutchinson_converged (Sec. III) for a block of probes
run together, with the target precision of Sec. VII.B and Sec. VIII.

Oracle, test infrastructure only.

The paper tests the Lanczos error of each probe and the error on the mean
separately and leaves the Lanczos error's estimate open.  This rule uses the
change of the block estimate over the last five steps as a crude stand-in
for the truncation error and combines it with the Hutchinson error:

  * after step j the block estimate is E_j = log2 T_j with T_j the mean over
    the probes of ||phi_n||^2 F_j,n (F_j,n the Gauss quadrature of |x| from
    T_j of probe n; a probe that broke down keeps its last value), and dE_j
    its error on the mean by the delta method (sample variance with N - 1);
  * the combined error is e_j = sqrt(dE_j^2 + (E_j - E_{j-5})^2), with dE_j
    taken as 0 when it is undefined (a single probe);
  * the first step that may stop is j = 6 (the first with an E_{j-5}); the
    run stops at the first j with e_j <= tol max(|E_j|, 1), else after the
    last step.  The estimate is E_j and its Lanczos part |E_j - E_{j-5}|.
"""
from __future__ import annotations

from typing import Dict

import numpy as np

FIRST_STEP = 6
LAG = 5


def block_estimate(beta: np.ndarray, F: np.ndarray, j: int) -> Dict[str, float]:
    """The plain block estimate after j steps: T = mean_n ||phi_n||^2 F_j,n,
    its standard error sqrt(Var / N) (N - 1 in the variance), E = log2 T
    (Eq. 1-2) and dE = SE / (T ln 2)."""
    G = np.asarray(beta, dtype=np.float64)[:, 0] ** 2 * np.asarray(F, dtype=np.float64)[:, j - 1]
    N = G.size
    T = float(np.mean(G))
    se = float(np.std(G, ddof=1) / np.sqrt(N)) if N > 1 else float("nan")
    return {"trace_norm": T, "trace_norm_se": se, "logneg": float(np.log2(T)),
            "logneg_se": se / (T * np.log(2.0)) if N > 1 else float("nan")}


def combined_error(beta: np.ndarray, F: np.ndarray, j: int) -> Dict[str, float]:
    """E_j, dE_j, the Lanczos proxy |E_j - E_{j-5}| and the combined error
    e_j (j >= 6)."""
    if j < FIRST_STEP:
        raise ValueError(f"the rule needs j >= {FIRST_STEP}")
    now = block_estimate(beta, F, j)
    old = block_estimate(beta, F, j - LAG)
    de = now["logneg_se"]
    dl = now["logneg"] - old["logneg"]
    err = float(np.sqrt((0.0 if np.isnan(de) else de * de) + dl * dl))
    return {"logneg": now["logneg"], "logneg_se": de, "lanczos_err": abs(dl), "err": err}


def stop_step(beta: np.ndarray, F: np.ndarray, tol: float) -> int:
    """First step j >= 6 whose combined error meets e_j <= tol max(|E_j|, 1),
    else the last step of the trajectories."""
    m = np.asarray(F).shape[1]
    for j in range(FIRST_STEP, m + 1):
        c = combined_error(beta, F, j)
        if np.isfinite(c["logneg"]) and c["err"] <= tol * max(abs(c["logneg"]), 1.0):
            return j
    return m


def run(beta: np.ndarray, F: np.ndarray, tol: float) -> Dict[str, float]:
    """The rule replayed on a block's trajectories: the stop step, the
    estimate there, its error on the mean and its Lanczos proxy (NaN before
    step 6)."""
    j = stop_step(beta, F, tol)
    est = block_estimate(beta, F, j)
    lerr = combined_error(beta, F, j)["lanczos_err"] if j >= FIRST_STEP else float("nan")
    return {"steps": j, "logneg": est["logneg"], "logneg_se": est["logneg_se"], "lanczos_err": lerr}
