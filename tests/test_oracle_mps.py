"""Pins for the matrix-product-state oracle (Sec. VI): the compressed
effective state must carry the nonzero spectrum of the full rho_AB^{T_B}."""
import numpy as np
import pytest

import tnslq_inputs as ti
from oracle import exact, mps

GEOMETRIES = [
    (12, 4, 2, 4, 6, 4),     # adjacent blocks
    (12, 4, 2, 4, 8, 3),     # gap of 2 sites, not compressed
    (12, 3, 0, 5, 5, 7),     # A at the left end, B at the right end
    (14, 4, 1, 5, 8, 6),     # B at the right end, gap 2
    (14, 2, 1, 3, 9, 3),     # gap of 5 sites compressed (2^5 > 2 x 2)
    (10, 8, 1, 3, 5, 3),
]


def _dense(ts, L, a0, LA, b0, LB):
    psi = mps.mps_to_dense(ts)
    psi = psi / np.linalg.norm(psi)
    return exact.regroup(psi, L, list(range(a0, a0 + LA)), list(range(b0, b0 + LB)))


def test_contraction_matches_a_direct_product():
    ts = ti.random_mps(5, 2, 3, 1)
    # psi[s0..s4] = M0[0,s0,:] M1[:,s1,:] ... M4[:,s4,0], written out for one index
    psi = mps.mps_to_dense(ts)
    s = (1, 0, 1, 1, 0)
    v = ts[0][:, s[0], :]
    for M, si in zip(ts[1:], s[1:]):
        v = v @ M[:, si, :]
    assert psi[int("".join(map(str, s)), 2)] == pytest.approx(v[0, 0], rel=1e-14)


@pytest.mark.parametrize("L,chi,a0,LA,b0,LB", GEOMETRIES)
def test_effective_state_keeps_the_partial_transpose_spectrum(L, chi, a0, LA, b0, LB):
    ts = ti.random_mps(L, 2, chi, L + chi)
    P = _dense(ts, L, a0, LA, b0, LB)
    Pe = mps.effective_state(ts, a0, LA, b0, LB)
    assert Pe.shape[0] * Pe.shape[1] <= P.shape[0] * P.shape[1]
    lam = np.sort(np.abs(exact.pt_spectrum(P)))[::-1]
    lam_e = np.sort(np.abs(exact.pt_spectrum(Pe)))[::-1]
    k = lam_e.size
    assert np.allclose(lam[:k], lam_e, atol=1e-13)
    assert np.all(lam[k:] < 1e-13)
    assert mps.logneg_mps_exact(ts, a0, LA, b0, LB) == pytest.approx(exact.logneg_exact(P), abs=1e-11)


def test_bell_pair_mps_has_one_bit_and_product_state_none():
    ts = ti.bell_pair_mps(10, 2, 7)
    assert mps.logneg_mps_exact(ts, 1, 3, 6, 3) == pytest.approx(1.0, abs=1e-12)
    # the pair inside A: nothing across the cut
    assert mps.logneg_mps_exact(ts, 1, 7, 8, 2) == pytest.approx(0.0, abs=1e-12)
    ts = ti.random_mps(10, 2, 1, 0)      # bond dimension 1: a product state
    assert mps.logneg_mps_exact(ts, 1, 3, 5, 4) == pytest.approx(0.0, abs=1e-12)


def test_semidefinite_cholesky():
    rng = np.random.default_rng(3)
    A = rng.standard_normal((6, 6)) + 1j * rng.standard_normal((6, 6))
    G = A @ A.conj().T
    # positive definite: the ordinary factor
    assert np.allclose(mps.psd_cholesky(G), np.linalg.cholesky(G), atol=1e-12)
    # rank 3 of 6: still G = L L^dagger, with zero columns
    B = A[:, :3]
    G3 = B @ B.conj().T
    Lr = mps.psd_cholesky(G3)
    assert np.allclose(Lr @ Lr.conj().T, G3, atol=1e-12)
    assert np.sum(np.any(np.abs(Lr) > 1e-9, axis=0)) == 3


def test_rank_deficient_gap_is_handled():
    # a Bell pair across a long gap: the gap's transfer matrix has rank 1
    ts = ti.bell_pair_mps(12, 2, 9)
    assert mps.logneg_mps_exact(ts, 1, 3, 7, 4) == pytest.approx(1.0, abs=1e-12)
