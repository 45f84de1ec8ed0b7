"""Logarithmic negativity of contiguous blocks of a matrix product state
(Sec. VI): a compressed form of rho_AB^{T_B} whose nonzero spectrum is that
of the full operator, reduced here to an effective dense state.

Oracle, test infrastructure only.

Conventions: an open-boundary MPS is a list of tensors M_i of shape
(chi_{i}, p_i, chi_{i+1}) with chi_0 = chi_L = 1 (Eq. 5 with the boundary bond
of size 1); psi's flat index has site 0 most significant.  A = sites
[a0, a0 + LA), B = sites [b0, b0 + LB) with a0 + LA <= b0 (gap g = b0 - a0 - LA).

The steps follow Sec. VI:
  * the sites left of A and right of B are traced out: their transfer
    products are positive matrices E_L (on the bond entering A) and E_R (on
    the bond leaving B); with E_L = X X^dagger and E_R = Y Y^dagger (Cholesky)
    the factors are absorbed into A and B, and their new bond indices u, v
    become environment indices traced between ket and bra (the gauge that
    removes the outer environments for open boundaries);
  * vertical decomposition of A (and B): when the section's physical space is
    larger than its bond space (p^LA > chi_u chi_m), the section S[u, a, m] is
    replaced by R[k, (u, m)] with R^dagger R = G, G[(u,m),(u',m')] =
    sum_a conj(S[u,a,m]) S[u',a,m'] (Cholesky): S = V R for an isometry V on
    the physical space, so rho_AB changes by an isometry on A (and on B, where
    the partial transpose turns it into its conjugate), which keeps the
    nonzero spectrum of rho^{T_B};
  * the gap section G[m, g, n] is traced: its transfer matrix, grouped as
    (m, n) against (m', n'), is positive, T = W W^dagger (Cholesky) when p^g
    exceeds chi_m chi_n, and W's column index becomes an environment index.
The effective state psi_eff[k_A, k_B, (u, w, v)] = sum_{m,n} R_A[k_A,u,m]
W[m,n,w] R_B[k_B,n,v], normalised, has rho_eff^{T_B} with the nonzero spectrum
of the state's rho_AB^{T_B}.
"""
from __future__ import annotations

from typing import List, Sequence

import numpy as np

from . import exact


def mps_to_dense(tensors: Sequence[np.ndarray]) -> np.ndarray:
    """Contract the chain into psi (flat, site 0 most significant)."""
    v = np.ones((1, 1), dtype=np.complex128)            # (flat physical so far, bond)
    for M in tensors:
        x, p, y = M.shape
        v = (v @ M.reshape(x, p * y)).reshape(-1, y)
    return v.reshape(-1)


def environment_left(tensors, a0: int) -> np.ndarray:
    """E_L[y, y'] = sum over sites < a0 of the ket/bra transfer product."""
    E = np.ones((1, 1), dtype=np.complex128)
    for M in tensors[:a0]:
        E = np.einsum("xz,xsy,zsw->yw", E, M, M.conj())
    return E


def environment_right(tensors, b1: int) -> np.ndarray:
    """E_R[x, x'] = sum over sites >= b1 of the ket/bra transfer product."""
    E = np.ones((1, 1), dtype=np.complex128)
    for M in reversed(tensors[b1:]):
        E = np.einsum("yw,xsy,zsw->xz", E, M, M.conj())
    return E


def section(tensors, i0: int, i1: int) -> np.ndarray:
    """S[x, phys, y]: the sites [i0, i1) contracted, phys with i0 most significant."""
    S = np.eye(tensors[i0].shape[0], dtype=np.complex128)[:, None, :]
    for M in tensors[i0:i1]:
        x, f, z = S.shape
        _, p, y = M.shape
        S = (S.reshape(x * f, z) @ M.reshape(z, p * y)).reshape(x, f * p, y)
    return S


def psd_cholesky(G: np.ndarray, tol: float = 1e-13) -> np.ndarray:
    """Lower Cholesky factor L of a positive semidefinite G (G = L L^dagger),
    column by column; a pivot not above tol times the largest diagonal entry
    leaves its column zero (the matrix is rank deficient there)."""
    G = np.asarray(G, dtype=np.complex128)
    n = G.shape[0]
    L = np.zeros_like(G)
    dmax = float(np.max(G.diagonal().real)) if n else 0.0
    for j in range(n):
        d = G[j, j].real - float(np.sum(np.abs(L[j, :j]) ** 2))
        if d > tol * dmax:
            L[j, j] = np.sqrt(d)
            L[j + 1:, j] = (G[j + 1:, j] - L[j + 1:, :j] @ L[j, :j].conj()) / L[j, j]
    return L


def _vertical(S: np.ndarray) -> np.ndarray:
    """R[k, u, m] with R^dagger R = sum_a conj(S[u,a,m]) S[u',a,m'] (or S itself
    as R[a, u, m] when the physical space is not larger than the bond space)."""
    u, a, m = S.shape
    if a <= u * m:
        return S.transpose(1, 0, 2)
    Sm = S.transpose(1, 0, 2).reshape(a, u * m)           # rows a, columns (u, m)
    G = Sm.conj().T @ Sm
    Lc = psd_cholesky(G)                                  # G = L L^dagger
    return Lc.conj().T.reshape(u * m, u, m)               # R = L^dagger


def effective_state(tensors, a0: int, LA: int, b0: int, LB: int) -> np.ndarray:
    """psi_eff of shape (d_A', d_B', d_E'), normalised (see module docstring)."""
    a1, b1 = a0 + LA, b0 + LB
    X = psd_cholesky(environment_left(tensors, a0))
    Y = psd_cholesky(environment_right(tensors, b1))
    SA = np.einsum("xu,xam->uam", X, section(tensors, a0, a1))
    SB = np.einsum("nby,yv->nbv", section(tensors, b0, b1), Y)
    RA = _vertical(SA)                                    # [kA, u, m]
    RB = _vertical(SB)                                    # [kB, n, v]
    if b0 == a1:
        W = np.eye(RA.shape[2], dtype=np.complex128)[:, :, None]      # m = n, w of size 1
    else:
        SG = section(tensors, a1, b0)                     # [m, g, n]
        m, g, n = SG.shape
        if g <= m * n:
            W = SG.transpose(0, 2, 1)                     # [m, n, w = g]
        else:
            Gm = SG.transpose(0, 2, 1).reshape(m * n, g)
            W = psd_cholesky(Gm @ Gm.conj().T).reshape(m, n, m * n)
    psi = np.einsum("aum,mnw,bnv->abuwv", RA, W, RB)
    dA, dB = RA.shape[0], RB.shape[0]
    psi = psi.reshape(dA, dB, -1)
    return psi / np.linalg.norm(psi)


def logneg_mps_exact(tensors, a0: int, LA: int, b0: int, LB: int) -> float:
    return exact.logneg_exact(effective_state(tensors, a0, LA, b0, LB))
