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


# ---------------------------------------------------------------- periodic
PERIODIC = [
    (8, 3, 0, 3, 3, 5),      # A and B cover the ring: the outer section is the identity
    (8, 3, 1, 3, 4, 3),      # adjacent, outer section of 2 sites (4 <= 9, not compressed)
    (10, 2, 1, 3, 5, 3),     # gap 1, outer section of 3 sites compressed (8 > 4)
    (10, 3, 2, 2, 6, 2),     # gap 2, outer section of 4 sites compressed (16 > 9)
    (12, 2, 2, 4, 7, 4),     # both blocks compressed (16 > 4), gap 1, outer of 3 sites
    (10, 2, 0, 4, 4, 6),     # blocks compressed, covering the ring
]


def test_periodic_contraction_is_a_trace_of_products():
    ts = ti.random_mps_periodic(5, 2, 3, 4)
    psi = mps.mps_to_dense(ts)
    s = (0, 1, 1, 0, 1)
    v = np.eye(3)
    for M, si in zip(ts, s):
        v = v @ M[:, si, :]
    assert psi[int("".join(map(str, s)), 2)] == pytest.approx(np.trace(v), rel=1e-14)


@pytest.mark.parametrize("L,chi,a0,LA,b0,LB", PERIODIC)
def test_periodic_effective_state_keeps_the_partial_transpose_spectrum(L, chi, a0, LA, b0, LB):
    ts = ti.random_mps_periodic(L, 2, chi, 3 * L + chi)
    P = _dense(ts, L, a0, LA, b0, LB)
    Pe = mps.effective_state(ts, a0, LA, b0, LB)
    lam = np.sort(np.abs(exact.pt_spectrum(P)))[::-1]
    lam_e = np.sort(np.abs(exact.pt_spectrum(Pe)))[::-1]
    k = min(lam.size, lam_e.size)
    assert np.allclose(lam[:k], lam_e[:k], atol=1e-13)
    assert np.all(lam[k:] < 1e-13) and np.all(lam_e[k:] < 1e-13)
    assert mps.logneg_mps_exact(ts, a0, LA, b0, LB) == pytest.approx(exact.logneg_exact(P), abs=1e-11)


def test_periodic_ring_with_a_closing_bond_of_one_is_the_open_chain():
    ts = ti.random_mps(10, 2, 4, 6)
    assert not mps.is_periodic(ts)
    assert mps.logneg_mps_exact(ts, 1, 3, 5, 4) == pytest.approx(
        exact.logneg_exact(_dense(ts, 10, 1, 3, 5, 4)), abs=1e-11)


# ------------------------------------------------- transfer-matrix route
@pytest.mark.parametrize("sites", [[2, 3, 4], [5], [7, 8, 9, 0, 1]])
def test_section_transfer_is_the_overlap_of_the_section(sites):
    ts = ti.random_mps_periodic(10, 2, 3, 8)
    S = mps.section_sites(ts, sites)
    want = np.einsum("xsy,zsw->xzwy", S, S.conj())
    got = mps.section_transfer(ts, sites)
    want = want / np.einsum("xxyy->", want).real
    assert np.allclose(got, want, atol=1e-14)
    # with a factor absorbed on the left bond
    X = np.tril(np.random.default_rng(1).standard_normal((3, 3))) + 3 * np.eye(3)
    SX = np.einsum("xu,xam->uam", X, S)
    want = np.einsum("xsy,zsw->xzwy", SX, SX.conj())
    got = mps.section_transfer(ts, sites, X)
    assert np.allclose(got, want / np.einsum("xxyy->", want).real, atol=1e-14)
    # the Gram matrix of the vertical decomposition is a regrouping of it
    Sm = SX.transpose(1, 0, 2).reshape(SX.shape[1], -1)
    G = Sm.conj().T @ Sm
    assert np.allclose(mps.gram_of_transfer(got), G / np.trace(G).real, atol=1e-14)


@pytest.mark.parametrize("L,chi,a0,LA,b0,LB", GEOMETRIES)
def test_transfer_route_gives_the_same_effective_state_open(L, chi, a0, LA, b0, LB):
    ts = ti.random_mps(L, 2, chi, L + chi)
    a = mps.effective_state(ts, a0, LA, b0, LB)
    b = mps.effective_state(ts, a0, LA, b0, LB, transfer=True)
    assert a.shape == b.shape
    assert np.max(np.abs(a - b)) <= 1e-11 * np.max(np.abs(a))


@pytest.mark.parametrize("L,chi,a0,LA,b0,LB", PERIODIC)
def test_transfer_route_gives_the_same_effective_state_periodic(L, chi, a0, LA, b0, LB):
    ts = ti.random_mps_periodic(L, 2, chi, 3 * L + chi)
    a = mps.effective_state(ts, a0, LA, b0, LB)
    b = mps.effective_state(ts, a0, LA, b0, LB, transfer=True)
    assert a.shape == b.shape
    assert np.max(np.abs(a - b)) <= 1e-11 * np.max(np.abs(a))


def _pair_logneg(c):
    # a pure two-qubit state with Schmidt coefficients sigma: E = 2 log2 sum sigma
    s = np.linalg.svd(c, compute_uv=False)
    return 2.0 * np.log2(np.sum(s))


def test_long_blocks_of_a_dimer_chain():
    # 80 sites, blocks of 30 and 34 sites (2^30 physical values: only the
    # transfer route reaches them); E is the pair cut by the A|B boundary
    ts, pairs = ti.dimer_mps(80, 11, offset=0)
    a0, LA, b0, LB = 5, 30, 35, 34        # boundary between sites 34 and 35
    cut = [c for (i, j), c in pairs if (i, j) == (34, 35)]
    assert len(cut) == 1
    assert mps.logneg_mps_exact(ts, a0, LA, b0, LB, transfer=True) == pytest.approx(_pair_logneg(cut[0]), abs=1e-12)
    # with a gap of one site no pair joins A and B
    assert mps.logneg_mps_exact(ts, a0, LA, b0 + 1, LB, transfer=True) == pytest.approx(0.0, abs=1e-12)


def test_long_blocks_of_a_dimer_ring():
    # the pair (79, 0) closes the ring: when A and B cover it both boundaries
    # cut a pair; when the outer section holds the closing pair only one does
    ts, pairs = ti.dimer_mps(80, 12, offset=1, periodic=True)
    assert mps.is_periodic(ts)
    c = dict(pairs)
    e_mid, e_wrap = _pair_logneg(c[(39, 40)]), _pair_logneg(c[(79, 0)])
    got = mps.logneg_mps_exact(ts, 0, 40, 40, 40, transfer=True)
    assert got == pytest.approx(e_mid + e_wrap, abs=1e-12)
    got = mps.logneg_mps_exact(ts, 1, 39, 40, 39, transfer=True)
    assert got == pytest.approx(e_mid, abs=1e-12)


@pytest.mark.parametrize("periodic", [True, False])
def test_ghz_blocks(periodic):
    # (|0..0> + |1..1>)/sqrt 2: one bit between two blocks covering the
    # chain, none once any site is traced
    ts = ti.ghz_mps(60, periodic)
    assert mps.logneg_mps_exact(ts, 0, 25, 25, 35, transfer=True) == pytest.approx(1.0, abs=1e-12)
    assert mps.logneg_mps_exact(ts, 0, 25, 26, 34, transfer=True) == pytest.approx(0.0, abs=1e-12)
    assert mps.logneg_mps_exact(ts, 3, 20, 23, 30, transfer=True) == pytest.approx(0.0, abs=1e-12)
