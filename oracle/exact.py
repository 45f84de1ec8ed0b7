"""Exact logarithmic negativity and the partial-transpose matvec.

Oracle, test infrastructure only.

Follows the plain definitions:
  * Sec. V: group psi's indices into subsystems A, B and C (= E, the rest),
    form the outer product with the conjugate, trace C, and swap the bra and
    ket indices of B;
  * Sec. II, Eq. 1: E(rho_AB) = log2 || rho_AB^{T_B} ||_Tr, the trace norm
    being the sum of |eigenvalues| of the Hermitian rho_AB^{T_B};
  * Sec. V, Eq. 4: (rho^{T_B} phi)_{ab} = sum_{a',b',c} psi_{ab'c} psi*_{a'bc} phi_{a'b'},
    both formed explicitly and contracted lazily through intermediary (i).

Conventions: qubit 0 is the most significant bit of the flat index; A and B
keep the order in which the partition lists them, C lists the remaining
qubits in increasing order.
"""
from __future__ import annotations

from typing import Sequence, Tuple

import numpy as np


def complement(n_qubits: int, a: Sequence[int], b: Sequence[int]) -> list:
    s = set(a) | set(b)
    return [q for q in range(n_qubits) if q not in s]


def regroup(psi: np.ndarray, n_qubits: int, a: Sequence[int], b: Sequence[int]) -> np.ndarray:
    """psi_{1..L} -> P[a, b, c] of shape (d_A, d_B, d_C) (Sec. V, Fig. 2(b))."""
    a, b = list(a), list(b)
    c = complement(n_qubits, a, b)
    t = np.asarray(psi, dtype=np.complex128).reshape([2] * n_qubits)
    t = np.transpose(t, a + b + c)
    return t.reshape(1 << len(a), 1 << len(b), 1 << len(c))


def regroup_dims(psi: np.ndarray, dims: Sequence[int], a: Sequence[int], b: Sequence[int]) -> np.ndarray:
    """The same for sites of any local dimension: psi's flat index in mixed
    radix over the sites (site 0 most significant, dims[s] values at site s);
    P[a, b, c] of shape (d_A, d_B, d_C) with a, b running over the listed sites
    in the given order and c over the other sites in increasing order."""
    a, b = list(a), list(b)
    c = complement(len(dims), a, b)
    t = np.asarray(psi, dtype=np.complex128).reshape(list(dims))
    t = np.transpose(t, a + b + c)
    d = lambda s: int(np.prod([dims[q] for q in s], dtype=np.int64))  # noqa: E731
    return t.reshape(d(a), d(b), d(c))


def rho_ab(P: np.ndarray) -> np.ndarray:
    """rho_AB[(a,b),(a',b')] = sum_c P[a,b,c] conj(P[a',b',c]) (Sec. V, Fig. 2(c))."""
    d_a, d_b, d_c = P.shape
    m = P.reshape(d_a * d_b, d_c)
    return m @ m.conj().T


def partial_transpose_b(rho: np.ndarray, d_a: int, d_b: int) -> np.ndarray:
    """rho^{T_B}[(a,b),(a',b')] = rho[(a,b'),(a',b)] (Sec. II; Sec. V, Fig. 2(d))."""
    r = rho.reshape(d_a, d_b, d_a, d_b)
    return r.transpose(0, 3, 2, 1).reshape(d_a * d_b, d_a * d_b)


def rho_pt(P: np.ndarray) -> np.ndarray:
    """The explicit operator rho_AB^{T_B} (intermediary (iii) of Sec. V)."""
    d_a, d_b, _ = P.shape
    return partial_transpose_b(rho_ab(P), d_a, d_b)


def pt_spectrum(P: np.ndarray) -> np.ndarray:
    """All eigenvalues of rho_AB^{T_B} (Sec. II: the full spectrum)."""
    return np.linalg.eigvalsh(rho_pt(P))


def trace_norm_exact(P: np.ndarray) -> float:
    """|| rho^{T_B} ||_Tr = sum |lambda_i| (Sec. II)."""
    return float(np.sum(np.abs(pt_spectrum(P))))


def logneg_exact(P: np.ndarray) -> float:
    """E = log2 || rho_AB^{T_B} ||_Tr (Sec. II, Eq. 1)."""
    return float(np.log2(trace_norm_exact(P)))


def logneg_of_state(psi: np.ndarray, n_qubits: int, a: Sequence[int], b: Sequence[int]) -> float:
    return logneg_exact(regroup(psi, n_qubits, a, b))


def pt_matvec_explicit(P: np.ndarray, X: np.ndarray) -> np.ndarray:
    """Y = rho^{T_B} X for a block X of shape (K, d_A*d_B), rows are vectors."""
    return (rho_pt(P) @ np.asarray(X, dtype=np.complex128).T).T


def pt_matvec_lazy(P: np.ndarray, X: np.ndarray) -> np.ndarray:
    """Y = rho^{T_B} X without forming rho (Sec. V, Eq. 4, intermediary (i)).

    For each probe k and environment index c:
        Upsilon[b', b] = sum_{a'} conj(P[a', b, c]) X_k[a', b']
        Y_k[a, b]     += sum_{b'} P[a, b', c] Upsilon[b', b]
    """
    d_a, d_b, d_c = P.shape
    X = np.asarray(X, dtype=np.complex128).reshape(-1, d_a, d_b)
    Y = np.zeros_like(X)
    for k in range(X.shape[0]):
        for c in range(d_c):
            m_c = np.ascontiguousarray(P[:, :, c])
            ups = X[k].T @ m_c.conj()          # (d_B x d_A)(d_A x d_B)
            Y[k] += m_c @ ups                  # (d_A x d_B)(d_B x d_B)
    return Y.reshape(X.shape[0], d_a * d_b)


def pt_matvec_bruteforce(P: np.ndarray, x: np.ndarray) -> np.ndarray:
    """Eq. 4 summed term by term in pure Python (tiny inputs only)."""
    d_a, d_b, d_c = P.shape
    x = np.asarray(x, dtype=np.complex128).reshape(d_a, d_b)
    y = np.zeros((d_a, d_b), dtype=np.complex128)
    for a in range(d_a):
        for b in range(d_b):
            s = 0.0j
            for a2 in range(d_a):
                for b2 in range(d_b):
                    for c in range(d_c):
                        s += P[a, b2, c] * np.conj(P[a2, b, c]) * x[a2, b2]
            y[a, b] = s
    return y.reshape(-1)


def purity_from_environment(P: np.ndarray) -> float:
    """Tr rho_AB^2 computed as Tr rho_C^2 from the d_C x d_C reduced matrix
    of the complement (the two are equal for a pure state)."""
    d_a, d_b, d_c = P.shape
    m = P.reshape(d_a * d_b, d_c)
    rho_c = m.T @ m.conj()
    return float(np.real(np.sum(rho_c * rho_c.T)))


def pt_matvec_entries_from_slabs(slab, d_c: int, x: np.ndarray, entries) -> np.ndarray:
    """Selected outputs y[a, b] of Eq. 4 for one vector x (d_A x d_B), for a
    state whose environment qubits are the leading ones, so that environment
    slab c is the d_A x d_B matrix slab(c) = psi[c, :, :] (A rows, B columns).

    For each c and each requested column b: u[b'] = sum_a' conj(M_c[a', b]) x[a', b'],
    then y[a, b] += sum_b' M_c[a, b'] u[b'].
    """
    x = np.asarray(x, dtype=np.complex128)
    entries = [(int(a), int(b)) for a, b in entries]
    cols = sorted({b for _, b in entries})
    y = np.zeros(len(entries), dtype=np.complex128)
    for c in range(d_c):
        m_c = slab(c)
        u = {b: np.conj(np.asarray(m_c[:, b], dtype=np.complex128)) @ x for b in cols}
        for t, (a, b) in enumerate(entries):
            y[t] += np.asarray(m_c[a, :], dtype=np.complex128) @ u[b]
    return y
