"""Pins for the oracle's exact logarithmic negativity and matvec (Sec. II,
Eq. 1; Sec. V, Eq. 4) against closed forms and brute force."""
import itertools

import numpy as np
import pytest

import tnslq_inputs as ti
from oracle import analytic, exact


def _le(psi, L, a, b):
    return exact.logneg_of_state(psi, L, a, b)


@pytest.mark.parametrize("bg", [None, 7])
def test_bell_pair_placements(bg):
    # Bell pair on qubits (1, 4) of 6 in a product background.
    L = 6
    psi = ti.bell_pair_state(L, 1, 4, background_seed=bg)
    assert _le(psi, L, [1], [4]) == pytest.approx(1.0, abs=1e-12)
    assert _le(psi, L, [0, 1, 2], [3, 4]) == pytest.approx(1.0, abs=1e-12)
    assert _le(psi, L, [4, 5], [1]) == pytest.approx(1.0, abs=1e-12)
    # both halves in A, or one half traced out: no entanglement between A and B
    assert _le(psi, L, [1, 4], [2, 3]) == pytest.approx(0.0, abs=1e-12)
    assert _le(psi, L, [1], [2, 3]) == pytest.approx(0.0, abs=1e-12)
    assert _le(psi, L, [0, 2], [3, 5]) == pytest.approx(0.0, abs=1e-12)


def test_product_states_have_zero_negativity():
    L = 7
    psi = ti.basis_product_state(L, [1, 0, 1, 1, 0, 0, 1])
    assert _le(psi, L, [0, 1], [4, 5, 6]) == pytest.approx(0.0, abs=1e-12)
    rng = np.random.default_rng(0)
    vec = np.array([1.0 + 0j])
    for _ in range(L):
        v = rng.standard_normal(2) + 1j * rng.standard_normal(2)
        vec = np.kron(vec, v / np.linalg.norm(v))
    assert _le(vec, L, [2, 0], [5, 3]) == pytest.approx(0.0, abs=1e-12)


def test_unit_trace_and_hermiticity():
    psi = ti.haar_state(9, 3)
    P = exact.regroup(psi, 9, [0, 4], [2, 7, 8])
    R = exact.rho_pt(P)
    assert np.trace(R) == pytest.approx(1.0, abs=1e-13)
    assert np.max(np.abs(R - R.conj().T)) < 1e-15


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_pure_state_reduces_to_schmidt_formula(seed):
    # Empty environment: E = 2 log2 sum_i sigma_i with sigma from an SVD of psi
    # as a d_A x d_B matrix, and the PT spectrum is {p_i} U {+-sqrt(p_i p_j)}_{i<j}.
    L, a, b = 6, [3, 0, 5], [1, 2, 4]
    psi = ti.haar_state(L, seed)
    M = psi.reshape([2] * L).transpose(a + b).reshape(8, 8)
    s = np.linalg.svd(M, compute_uv=False)
    assert _le(psi, L, a, b) == pytest.approx(2 * np.log2(np.sum(s)), abs=1e-12)
    p = s ** 2
    spec = list(p)
    for i, j in itertools.combinations(range(len(p)), 2):
        r = np.sqrt(p[i] * p[j])
        spec += [r, -r]
    P = exact.regroup(psi, L, a, b)
    assert np.allclose(np.sort(exact.pt_spectrum(P)), np.sort(spec), atol=1e-14)


def test_frobenius_norm_equals_environment_purity():
    # ||rho^{T_B}||_F^2 = Tr rho_AB^2 = Tr rho_C^2 (Sec. VIII Eq. 10; pure state)
    psi = ti.haar_state(10, 4)
    P = exact.regroup(psi, 10, [1, 2, 3], [6, 8])
    R = exact.rho_pt(P)
    lhs = float(np.real(np.sum(R * R.conj())))
    assert lhs == pytest.approx(exact.purity_from_environment(P), rel=1e-12)
    assert lhs == pytest.approx(float(np.sum(exact.pt_spectrum(P) ** 2)), rel=1e-12)


def test_matvec_matches_bruteforce_eq4():
    psi = ti.haar_state(6, 9)
    P = exact.regroup(psi, 6, [4, 1], [0, 5])
    rng = np.random.default_rng(1)
    x = rng.standard_normal(16) + 1j * rng.standard_normal(16)
    y_bf = exact.pt_matvec_bruteforce(P, x)
    assert np.allclose(exact.pt_matvec_explicit(P, x[None])[0], y_bf, atol=1e-15)
    assert np.allclose(exact.pt_matvec_lazy(P, x[None])[0], y_bf, atol=1e-15)


def test_ab_symmetry_and_ordering_invariance():
    L = 9
    psi = ti.haar_state(L, 5)
    e0 = _le(psi, L, [0, 3, 4], [6, 7])
    assert _le(psi, L, [6, 7], [0, 3, 4]) == pytest.approx(e0, abs=1e-12)
    assert _le(psi, L, [4, 0, 3], [7, 6]) == pytest.approx(e0, abs=1e-12)


def test_local_unitary_invariance():
    L = 8
    psi = ti.haar_state(L, 6)
    a, b = [0, 1, 5], [2, 6]
    e0 = _le(psi, L, a, b)
    rng = np.random.default_rng(3)
    t = psi.reshape([2] * L)
    for q in range(L):
        u = ti.haar_unitary(2, rng)
        t = np.moveaxis(np.tensordot(u, t, axes=([1], [q])), 0, q)
    assert _le(t.reshape(-1), L, a, b) == pytest.approx(e0, abs=1e-12)


def _pair_logneg(u):
    # pure two-qubit state U|00>: E = 2 log2 (sigma_0 + sigma_1)
    s = np.linalg.svd(u[:, 0].reshape(2, 2), compute_uv=False)
    return 2 * np.log2(np.sum(s))


def test_depth_one_brickwork_factorises_over_gates():
    L, seed = 8, 2
    gates = ti.brickwork_gates(L, 1, seed)        # pairs (0,1), (2,3), (4,5), (6,7)
    psi = ti.brickwork_state(L, 1, seed)
    # A = {1, 2}, B = {0, 3, 4}: gates (0,1) and (2,3) straddle A|B, (4,5) is B|E
    want = _pair_logneg(gates[0][1]) + _pair_logneg(gates[1][1])
    assert _le(psi, L, [1, 2], [0, 3, 4]) == pytest.approx(want, abs=1e-12)
    # no A-B pair at depth one: exactly zero (the brickwork sweep's partition shape)
    L = 12
    psi = ti.brickwork_state(L, 1, 1)
    assert _le(psi, L, [2, 3, 4, 5], [7, 8, 9]) == pytest.approx(0.0, abs=1e-12)


def test_random_state_formula_eq6():
    assert analytic.random_state_logneg(4, 4, 64) == 0.0         # R = 1
    assert analytic.random_state_logneg(2, 2, 64) == 0.0         # R < 1
    # large-d limit: a 16-qubit Haar state, |A| = |B| = 5, |C| = 6 (R = 8)
    L = 16
    psi = ti.haar_state(L, 0)
    e = _le(psi, L, list(range(5)), list(range(5, 10)))
    want = analytic.random_state_logneg(32, 32, 64)
    assert abs(e - want) < 0.02 * want


def test_sampled_entries_match_explicit_matvec():
    # environment = the leading qubits, so slab c is psi[c] as a d_A x d_B matrix
    L = 8
    psi = ti.haar_state(L, 12)
    a, b = [2, 3, 4], [5, 6, 7]
    P = exact.regroup(psi, L, a, b)
    x = ti.random_vectors(1, 64, seed=2)
    y = exact.pt_matvec_explicit(P, x)[0].reshape(8, 8)
    slab = lambda c: psi.reshape(4, 8, 8)[c]  # noqa: E731
    entries = [(0, 3), (5, 3), (7, 0), (2, 6)]
    got = exact.pt_matvec_entries_from_slabs(slab, 4, x[0].reshape(8, 8), entries)
    assert np.allclose(got, [y[i, j] for i, j in entries], atol=1e-15)
