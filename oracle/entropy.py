"""Other spectral sums by the same method: von Neumann entropy and purity of a
subsystem, and the mutual information (the paper's closing section: the same
stochastic Lanczos quadrature applies to other functions of reduced density
matrices, with the partial transpose dropped).

Oracle, test infrastructure only.

Definitions (pure state psi on L qubits, subsystem S, rest R):
  Psi      psi regrouped as a d_S x d_R matrix (S's qubits in the given order,
           most significant first; R the remaining qubits in increasing order)
  rho_S    = Tr_R |psi><psi| = Psi Psi^dagger
  S(S)     = -Tr rho_S log2 rho_S = -sum_i p_i log2 p_i   (0 log 0 = 0)
  purity   = Tr rho_S^2 = sum_i p_i^2
  I(A:B)   = S(A) + S(B) - S(AB), and S(AB) = S(E) for a pure global state
with p_i the eigenvalues of rho_S, the squared singular values of Psi
(Schmidt coefficients).  rho_S and rho_R have the same non-zero spectrum.

Stochastic estimate: Algorithm 1 with the operator rho_S, applied lazily as
rho_S X = Psi (Psi^dagger X), and f(x) = -x log2 x (taken as 0 for x <= 0:
Ritz values of a positive semi-definite operator can come out at -1e-17) or
f(x) = x^2.  The estimate is the Hutchinson mean itself, G_n = ||phi_n||^2 F_m
(no logarithm), with its error on the mean.

Reading: the operator is built on the smaller side; when d_S > d_R the
Krylov space is that of rho_R, which has the same spectral sums.
"""
from __future__ import annotations

from typing import Dict, Sequence

import numpy as np

from . import exact, probes, slq


def bipartition(n_qubits: int, s: Sequence[int]):
    """(S, R) with R the complement of S in increasing order."""
    s = list(s)
    return s, exact.complement(n_qubits, s, [])


def psi_matrix(psi: np.ndarray, n_qubits: int, s: Sequence[int]) -> np.ndarray:
    """Psi[s, r] of shape (d_S, d_R)."""
    P = exact.regroup(psi, n_qubits, s, [])
    return P.reshape(P.shape[0], P.shape[2])


def operator_side(n_qubits: int, s: Sequence[int]):
    """The side whose reduced density matrix carries the Krylov space: the
    smaller of S and its complement (S when equal)."""
    s, r = bipartition(n_qubits, s)
    return s if len(s) <= len(r) else r


def schmidt_probabilities(psi: np.ndarray, n_qubits: int, s: Sequence[int]) -> np.ndarray:
    sig = np.linalg.svd(psi_matrix(psi, n_qubits, s), compute_uv=False)
    return sig * sig


def f_entropy(x):
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros_like(x)
    pos = x > 0
    out[pos] = -x[pos] * np.log2(x[pos])
    return out


def f_purity(x):
    x = np.asarray(x, dtype=np.float64)
    return x * x


FUNCTIONS = {"entropy": f_entropy, "purity": f_purity}


def entropy_exact(psi: np.ndarray, n_qubits: int, s: Sequence[int]) -> float:
    return float(np.sum(f_entropy(schmidt_probabilities(psi, n_qubits, s))))


def purity_exact(psi: np.ndarray, n_qubits: int, s: Sequence[int]) -> float:
    return float(np.sum(f_purity(schmidt_probabilities(psi, n_qubits, s))))


def mutual_information_exact(psi: np.ndarray, n_qubits: int, a: Sequence[int], b: Sequence[int]) -> float:
    return (entropy_exact(psi, n_qubits, a) + entropy_exact(psi, n_qubits, b)
            - entropy_exact(psi, n_qubits, list(a) + list(b)))


def reduced_density_matrix(psi: np.ndarray, n_qubits: int, s: Sequence[int]) -> np.ndarray:
    M = psi_matrix(psi, n_qubits, s)
    return M @ M.conj().T


def rho_matvec(M: np.ndarray, X: np.ndarray) -> np.ndarray:
    """rows of Y = rho X^T for rho = M M^dagger, as two products over M."""
    Z = M.conj().T @ X.T
    return (M @ Z).T


def slq_spectral_sum(psi: np.ndarray, n_qubits: int, s: Sequence[int], fn: str, n_probes: int, n_steps: int,
                     seed: int, probe_offset: int = 0, reorth: bool = False) -> Dict[str, object]:
    """Algorithm 1 on rho of the operator side with f = FUNCTIONS[fn]; the
    estimate of Tr f(rho_S) is the mean of G_n."""
    side = operator_side(n_qubits, s)
    M = psi_matrix(psi, n_qubits, side)
    X = probes.rademacher_probes(seed, n_probes, M.shape[0], probe_offset)
    r = slq.slq(lambda v: rho_matvec(M, v[None, :])[0], X, n_steps, reorth, FUNCTIONS[fn])
    r["value"] = r["trace_norm"]
    r["value_se"] = r["trace_norm_se"]
    r["side"] = side
    return r


def page_entropy(d_s: int, d_r: int) -> float:
    """Page's mean entanglement entropy of a Haar-random pure state, in bits
    (d_s <= d_r): sum_{k=d_r+1}^{d_s d_r} 1/k - (d_s - 1) / (2 d_r), in nats."""
    if d_s > d_r:
        d_s, d_r = d_r, d_s
    k = np.arange(d_r + 1, d_s * d_r + 1, dtype=np.float64)
    return float((np.sum(1.0 / k) - (d_s - 1) / (2.0 * d_r)) / np.log(2.0))


def haar_mean_purity(d_s: int, d_r: int) -> float:
    """Mean purity of a Haar-random pure state: (d_s + d_r) / (d_s d_r + 1)."""
    return (d_s + d_r) / (d_s * d_r + 1.0)
