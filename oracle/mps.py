"""Logarithmic negativity of contiguous blocks of a matrix product state
(Sec. VI): a compressed form of rho_AB^{T_B} whose nonzero spectrum is that
of the full operator, reduced here to an effective dense state.

Oracle, test infrastructure only.

Conventions: site i holds M_i of shape (chi_i, p_i, chi_{i+1}) (Eq. 5); psi's
flat index has site 0 most significant.  Open boundaries: chi_0 = chi_L = 1.
Periodic boundaries: chi_0 = chi_L > 1 and psi = Tr(M_0 ... M_{L-1}) (the
closing bond summed; Fig. 4(b)).  A = sites [a0, a0 + LA), B = sites
[b0, b0 + LB) with a0 + LA <= b0 (gap g = b0 - a0 - LA).  Bonds: u enters A,
m leaves A, n enters B, v leaves B.

The steps follow Sec. VI:
  * open boundaries: the sites left of A and right of B are traced out; their
    transfer products are positive matrices E_L (on u) and E_R (on v); with
    E_L = X X^dagger and E_R = Y Y^dagger (Cholesky) the factors are absorbed
    into A and B, and u, v become environment indices traced between ket and
    bra (the gauge that removes the outer environments);
  * periodic boundaries: the sites right of B and left of A form one section
    O[v, o, u] that closes the ring through the boundary bond (identity
    delta(v, u) when A and B cover the ring); it is traced like the gap below,
    Z Z^dagger = its transfer matrix grouped as (v, u) against (v', u'), and
    Z's column index z joins the environment;
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
The effective state, normalised, is
  open:      psi_eff[k_A, k_B, (u, w, v)] = sum_{m,n} R_A[k_A,u,m] W[m,n,w] R_B[k_B,n,v],
  periodic:  psi_eff[k_A, k_B, (w, z)] = sum_{u,m,n,v} R_A[k_A,u,m] W[m,n,w] R_B[k_B,n,v] Z[v,u,z],
and rho_eff^{T_B} has the nonzero spectrum of the state's rho_AB^{T_B}.

Two ways to the matrices that are factored (`transfer`):
  * False: every section is contracted explicitly (its physical index whole),
    and the Gram matrices are products over that index;
  * True: a compressed section's transfer matrix (the first step of Sec. VI's
    lateral compression: the section's overlap with its conjugate over the
    physical indices, as a chi^2 x chi^2 object) is built site by site, so
    blocks and gaps of any length cost chi^5 p per site; the Gram matrix of
    the vertical decomposition and the gap's matrix are that same tensor with
    its four bond axes regrouped.  The trimming of small singular values in
    that step is not taken: it would leave the regrouped matrices indefinite
    (the factors are exact here).
"""
from __future__ import annotations

from typing import List, Optional, Sequence

import numpy as np

from . import exact


def is_periodic(tensors) -> bool:
    """A chain whose boundary bond is wider than 1 is periodic (chi_0 = chi_L)."""
    c0, cL = tensors[0].shape[0], tensors[-1].shape[2]
    if c0 != cL:
        raise ValueError("boundary bonds differ: chi_0 = %d, chi_L = %d" % (c0, cL))
    return c0 > 1


def section_sites(tensors, sites: Sequence[int]) -> np.ndarray:
    """S[x, phys, y]: the listed sites contracted in order (consecutive along
    the ring), phys with the first site most significant."""
    sites = list(sites)
    S = np.eye(tensors[sites[0]].shape[0], dtype=np.complex128)[:, None, :]
    for i in sites:
        M = tensors[i]
        x, f, z = S.shape
        _, p, y = M.shape
        S = (S.reshape(x * f, z) @ M.reshape(z, p * y)).reshape(x, f * p, y)
    return S


def section(tensors, i0: int, i1: int) -> np.ndarray:
    """S[x, phys, y]: the sites [i0, i1) contracted, phys with i0 most significant."""
    return section_sites(tensors, range(i0, i1))


def mps_to_dense(tensors: Sequence[np.ndarray]) -> np.ndarray:
    """Contract the chain into psi (flat, site 0 most significant); the
    boundary bond is traced (size 1 for open boundaries)."""
    is_periodic(tensors)
    S = section(tensors, 0, len(tensors))
    return np.einsum("xsx->s", S)


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


def section_transfer(tensors, sites: Sequence[int], X: Optional[np.ndarray] = None) -> np.ndarray:
    """T[x, x', y', y] = sum_s S[x, s, y] conj(S[x', s, y']) for the section S
    over `sites` (with X absorbed on its left bond, S -> X^T S, when given),
    one site at a time: T <- sum_{z, z', s} T[x, x', z', z] M[z, s, y]
    conj(M[z', s, y']).  Each step divides by the trace sum_{x, y}
    T[x, x, y, y] (a positive scale; the effective state is normalised at
    the end)."""
    sites = list(sites)
    chi = tensors[sites[0]].shape[0]
    if X is None:
        X = np.eye(chi, dtype=np.complex128)
    T = np.einsum("zu,wv->uvwz", X, X.conj())
    T = T / np.einsum("xxyy->", T).real
    for i in sites:
        M = tensors[i]
        T = np.einsum("abqz,zsy,qsw->abwy", T, M, M.conj(), optimize=True)
        T = T / np.einsum("xxyy->", T).real
    return T


def absorb_right(T: np.ndarray, Y: np.ndarray) -> np.ndarray:
    """The transfer matrix of S -> S Y: T'[x, x', v', v] = sum conj(Y[y', v'])
    T[x, x', y', y] Y[y, v]."""
    return np.einsum("abqz,qw,zv->abwv", T, Y.conj(), Y, optimize=True)


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


def gram_of_transfer(T: np.ndarray) -> np.ndarray:
    """G[(x, y), (x', y')] = sum_s conj(S[x,s,y]) S[x',s,y'] = T[x', x, y, y']."""
    x, _, y, _ = T.shape
    return T.transpose(1, 2, 0, 3).reshape(x * y, x * y)


def _vertical_transfer(T: np.ndarray) -> np.ndarray:
    """R[k, x, y] = L^dagger for the Gram matrix of a section given by its
    transfer matrix T[x, x', y', y] (the same R as _vertical)."""
    x, _, y, _ = T.shape
    return psd_cholesky(gram_of_transfer(T)).conj().T.reshape(x * y, x, y)


def trace_factor_of_transfer(T: np.ndarray) -> np.ndarray:
    """F[x, y, f] with sum_f F[x,y,f] conj(F[x',y',f]) = sum_s S[x,s,y]
    conj(S[x',s,y']) = T[x, x', y', y] grouped as (x, y) against (x', y')."""
    x, _, y, _ = T.shape
    return psd_cholesky(T.transpose(0, 3, 1, 2).reshape(x * y, x * y)).reshape(x, y, x * y)


def _trace_factor(S: np.ndarray) -> np.ndarray:
    """F[x, y, f] for an explicit section S[x, g, y]: S itself as F[x, y, g]
    when its physical space is not larger than x y, else the Cholesky factor
    of sum_g S[x,g,y] conj(S[x',g,y'])."""
    x, g, y = S.shape
    if g <= x * y:
        return S.transpose(0, 2, 1)
    Sm = S.transpose(0, 2, 1).reshape(x * y, g)
    return psd_cholesky(Sm @ Sm.conj().T).reshape(x, y, x * y)


def _physical_size(tensors, sites) -> int:
    n = 1
    for i in sites:
        n *= int(tensors[i].shape[1])
    return n


def effective_state(tensors, a0: int, LA: int, b0: int, LB: int, transfer: bool = False) -> np.ndarray:
    """psi_eff of shape (d_A', d_B', d_E'), normalised (see module docstring)."""
    L = len(tensors)
    a1, b1 = a0 + LA, b0 + LB
    closed = is_periodic(tensors)
    U, Mb = tensors[a0].shape[0], tensors[a1 - 1].shape[2]
    Nb, V = tensors[b0].shape[0], tensors[b1 - 1].shape[2]
    X = Y = None
    if not closed:
        X = psd_cholesky(environment_left(tensors, a0))
        Y = psd_cholesky(environment_right(tensors, b1))
    sitesA, sitesB = range(a0, a1), range(b0, b1)
    # block A: R_A[kA, u, m]
    if transfer and _physical_size(tensors, sitesA) > U * Mb:
        RA = _vertical_transfer(section_transfer(tensors, sitesA, X))
    else:
        SA = section(tensors, a0, a1)
        RA = _vertical(SA if X is None else np.einsum("xu,xam->uam", X, SA))
    # block B: R_B[kB, n, v]
    if transfer and _physical_size(tensors, sitesB) > Nb * V:
        TB = section_transfer(tensors, sitesB)
        RB = _vertical_transfer(TB if Y is None else absorb_right(TB, Y))
    else:
        SB = section(tensors, b0, b1)
        RB = _vertical(SB if Y is None else np.einsum("nby,yv->nbv", SB, Y))
    # the gap: W[m, n, w]
    if b0 == a1:
        W = np.eye(Mb, dtype=np.complex128)[:, :, None]      # m = n, w of size 1
    elif transfer and _physical_size(tensors, range(a1, b0)) > Mb * Nb:
        W = trace_factor_of_transfer(section_transfer(tensors, range(a1, b0)))
    else:
        W = _trace_factor(section(tensors, a1, b0))
    if not closed:
        psi = np.einsum("aum,mnw,bnv->abuwv", RA, W, RB)
    else:
        # the outer section closing the ring: Z[v, u, z]
        sitesO = list(range(b1, L)) + list(range(0, a0))
        if not sitesO:
            Z = np.eye(V, dtype=np.complex128)[:, :, None]
        elif transfer and _physical_size(tensors, sitesO) > V * U:
            Z = trace_factor_of_transfer(section_transfer(tensors, sitesO))
        else:
            Z = _trace_factor(section_sites(tensors, sitesO))
        psi = np.einsum("aum,mnw,bnv,vuz->abwz", RA, W, RB, Z)
    dA, dB = RA.shape[0], RB.shape[0]
    psi = psi.reshape(dA, dB, -1)
    return psi / np.linalg.norm(psi)


def logneg_mps_exact(tensors, a0: int, LA: int, b0: int, LB: int, transfer: bool = False) -> float:
    return exact.logneg_exact(effective_state(tensors, a0, LA, b0, LB, transfer))
