"""Stochastic Lanczos quadrature (Sec. III, Algorithm 1) and its error bar
(Sec. VIII).

Oracle, test infrastructure only.

What is computed, per probe vector phi: the Lanczos process on the Hermitian
operator started from phi / ||phi|| builds, one matvec per step, the
tridiagonal matrix T_k of the operator restricted to the Krylov space (its
diagonal alpha from the Rayleigh quotients of the basis vectors, its
off-diagonal beta from the norms of the orthogonalised remainders).  The
Gauss quadrature of f on the probe's spectral measure is then the sum over
the eigenpairs of T_k of f(eigenvalue) weighted by the squared first
component of the eigenvector.  Hutchinson's estimator averages
||phi||^2 times that quadrature over independent probes; E = log2 of the
mean for f = |x| (Eq. 1-2), with the error on the mean of Sec. VIII.

Readings where the paper is silent (each also listed in the design notes):
  * the quadrature estimates the bilinear form for the *normalised* start
    vector; Hutchinson's sum needs <phi|f|phi>, hence the factor ||phi||^2
    (= beta_1^2) in G_n;
  * the diagonal coefficient is the real part of <q_k | X q_k> (the operator
    is Hermitian);
  * lanczos_estimate is the quadrature after a fixed number m of steps (no
    early exit);
  * breakdown: a probe stops when beta_{k+1} <= 1e-12 * s_k with
    s_k = max_{i<=k} |alpha_i| + max_{2<=i<=k} beta_i; the quadrature of
    T_k is then exact and later quadrature values repeat it;
  * reorthogonalisation (when asked for) is classical Gram-Schmidt applied
    twice against every earlier Lanczos vector of the same probe;
  * the error on the mean uses the sample variance with N-1 in the
    denominator; the error of E follows by the delta method,
    dE = SE / (mean * ln 2).
"""
from __future__ import annotations

from typing import Callable, Dict, Optional

import numpy as np
import scipy.linalg

from . import exact, probes

BREAKDOWN_TOL = 1e-12


def lanczos(matvec: Callable[[np.ndarray], np.ndarray], phi: np.ndarray, m: int,
            reorth: bool = False):
    """Lanczos recurrence of Algorithm 1 for one probe.

    Returns (alpha[m], beta[m+1], steps): beta[0] = beta_1 = ||phi||,
    beta[k] = beta_{k+1}; entries past a breakdown are zero.
    """
    phi = np.asarray(phi, dtype=np.complex128)
    alpha = np.zeros(m)
    beta = np.zeros(m + 1)
    beta[0] = np.linalg.norm(phi)
    q_prev = np.zeros_like(phi)
    q = phi / beta[0]
    basis = [q]
    amax = 0.0
    bmax = 0.0
    steps = 0
    for k in range(m):
        v = matvec(q) - beta[k] * q_prev if k > 0 else matvec(q)
        alpha[k] = np.real(np.vdot(q, v))
        v = v - alpha[k] * q
        if reorth:
            Q = np.array(basis)
            for _ in range(2):
                v = v - Q.T @ (Q.conj() @ v)
        beta[k + 1] = np.linalg.norm(v)
        steps = k + 1
        amax = max(amax, abs(alpha[k]))
        if k > 0:
            bmax = max(bmax, beta[k])
        if beta[k + 1] <= BREAKDOWN_TOL * (amax + bmax):
            break
        q_prev, q = q, v / beta[k + 1]
        basis.append(q)
    return alpha, beta, steps


def gauss_quadrature(alpha: np.ndarray, beta_off: np.ndarray,
                     f: Callable[[np.ndarray], np.ndarray] = np.abs) -> float:
    """F = sum_j tau_j^2 f(theta_j) for T = tridiag(alpha; beta_off)
    (Algorithm 1, the quadrature block): theta, w from the eigensystem of T,
    tau_j the first component of w_j."""
    alpha = np.asarray(alpha, dtype=np.float64)
    if alpha.size == 1:
        return float(f(alpha)[0])
    theta, w = scipy.linalg.eigh_tridiagonal(alpha, np.asarray(beta_off, dtype=np.float64))
    tau = w[0, :]
    return float(np.sum(tau * tau * f(theta)))


def quadrature_trajectory(alpha: np.ndarray, beta: np.ndarray, steps: int,
                          f: Callable[[np.ndarray], np.ndarray] = np.abs) -> np.ndarray:
    """[F_1, ..., F_m] for one probe; F_k for k > steps repeats F_steps."""
    m = alpha.size
    out = np.zeros(m)
    for k in range(1, m + 1):
        kk = min(k, steps)
        out[k - 1] = gauss_quadrature(alpha[:kk], beta[1:kk], f)
    return out


def hutchinson_stats(G: np.ndarray) -> Dict[str, float]:
    """Mean, standard error sqrt(Var/N) (Sec. VIII), E = log2(mean) (Eq. 2)
    and its delta-method error."""
    G = np.asarray(G, dtype=np.float64)
    n = G.size
    mean = float(np.mean(G))
    se = float(np.std(G, ddof=1) / np.sqrt(n)) if n > 1 else float("nan")
    e = float(np.log2(mean))
    de = se / (mean * np.log(2.0)) if n > 1 else float("nan")
    return {"trace_norm": mean, "trace_norm_se": se, "logneg": e, "logneg_se": de}


def slq(matvec: Callable[[np.ndarray], np.ndarray], probe_block: np.ndarray, m: int,
        reorth: bool = False, f: Callable[[np.ndarray], np.ndarray] = np.abs) -> Dict[str, object]:
    """Algorithm 1 with fixed N = len(probe_block) and K_max = m."""
    K, n = probe_block.shape
    alpha = np.zeros((K, m))
    beta = np.zeros((K, m + 1))
    steps = np.zeros(K, dtype=np.int64)
    F = np.zeros((K, m))
    G = np.zeros(K)
    for k in range(K):
        a, b, s = lanczos(matvec, probe_block[k], m, reorth)
        alpha[k], beta[k], steps[k] = a, b, s
        F[k] = quadrature_trajectory(a, b, s, f)
        G[k] = b[0] ** 2 * F[k, -1]
    out = {"alpha": alpha, "beta": beta, "steps": steps, "F": F, "G": G}
    out.update(hutchinson_stats(G))
    return out


def slq_logneg(psi: np.ndarray, n_qubits: int, a, b, n_probes: int, n_steps: int, seed: int,
               probe_offset: int = 0, reorth: bool = False, matvec: str = "explicit",
               ) -> Dict[str, object]:
    """SLQ estimate of log2 Tr|rho_AB^{T_B}| on the seeded probes of ``probes``."""
    P = exact.regroup(psi, n_qubits, a, b)
    d_a, d_b, _ = P.shape
    if matvec == "explicit":
        R = exact.rho_pt(P)
        mv = lambda v: R @ v  # noqa: E731
    else:
        mv = lambda v: exact.pt_matvec_lazy(P, v[None, :])[0]  # noqa: E731
    X = probes.rademacher_probes(seed, n_probes, d_a * d_b, probe_offset)
    return slq(mv, X, n_steps, reorth)


def slq_logneg_dims(psi: np.ndarray, dims, a, b, n_probes: int, n_steps: int, seed: int, probe_offset: int = 0,
                    reorth: bool = False) -> Dict[str, object]:
    """slq_logneg for sites of any local dimension (explicit operator)."""
    P = exact.regroup_dims(psi, dims, a, b)
    R = exact.rho_pt(P)
    X = probes.rademacher_probes(seed, n_probes, P.shape[0] * P.shape[1], probe_offset)
    return slq(lambda v: R @ v, X, n_steps, reorth)
