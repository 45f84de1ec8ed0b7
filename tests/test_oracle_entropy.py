"""Pins for the entropy / purity / mutual-information oracle."""
import numpy as np
import pytest
import scipy.linalg

import tnslq_inputs as ti
from oracle import entropy as en
from oracle import exact, probes


def _bell_times_bell(L, p1, p2):
    """Two Bell pairs on qubit pairs p1, p2, the other qubits |0>."""
    t = np.zeros([2] * L, dtype=np.complex128)
    for x in (0, 1):
        for y in (0, 1):
            idx = [0] * L
            idx[p1[0]] = idx[p1[1]] = x
            idx[p2[0]] = idx[p2[1]] = y
            t[tuple(idx)] = 0.5
    return t.reshape(-1)


def test_bell_pair_has_one_bit_and_purity_half():
    psi = ti.bell_pair_state(6, 1, 4)
    assert en.entropy_exact(psi, 6, [0, 1, 2]) == pytest.approx(1.0, abs=1e-14)
    assert en.purity_exact(psi, 6, [0, 1, 2]) == pytest.approx(0.5, abs=1e-14)
    # both qubits of the pair on one side: no entanglement across the cut
    assert en.entropy_exact(psi, 6, [0, 1, 4]) == pytest.approx(0.0, abs=1e-14)


def test_product_state_is_pure():
    psi = ti.basis_product_state(7, [1, 0, 1, 1, 0, 0, 1])
    assert en.entropy_exact(psi, 7, [2, 5]) == pytest.approx(0.0, abs=1e-14)
    assert en.purity_exact(psi, 7, [2, 5]) == pytest.approx(1.0, abs=1e-14)


def test_ghz_single_qubit_entropy():
    psi = np.zeros(8, dtype=np.complex128)
    psi[0] = psi[7] = 2 ** -0.5
    assert en.entropy_exact(psi, 3, [1]) == pytest.approx(1.0, abs=1e-14)
    assert en.entropy_exact(psi, 3, [0, 2]) == pytest.approx(1.0, abs=1e-14)


def test_mutual_information_counts_shared_pairs():
    # pair (0, 3) shared by A = {0, 1} and B = {2, 3}; pair (1, 5) ties A to E:
    # S(A) = 2, S(B) = 1, S(AB) = S(E) = 1, so I(A:B) = 2
    psi = _bell_times_bell(6, (0, 3), (1, 5))
    assert en.mutual_information_exact(psi, 6, [0, 1], [2, 3]) == pytest.approx(2.0, abs=1e-13)


def test_schmidt_route_matches_eigensolver_and_complement():
    L = 9
    psi = ti.haar_state(L, 3)
    for s in ([0, 4, 7], [2], [1, 2, 3, 5, 8]):
        rho = en.reduced_density_matrix(psi, L, s)
        lam = scipy.linalg.eigvalsh(rho)
        want = float(np.sum(en.f_entropy(np.clip(lam, 0, None))))
        assert en.entropy_exact(psi, L, s) == pytest.approx(want, abs=1e-12)
        assert en.purity_exact(psi, L, s) == pytest.approx(float(np.sum(lam * lam)), rel=1e-12)
        r = exact.complement(L, s, [])
        assert en.entropy_exact(psi, L, r) == pytest.approx(en.entropy_exact(psi, L, s), abs=1e-12)


def test_haar_state_matches_page_and_mean_purity():
    L, s = 14, list(range(6))
    vals = [en.entropy_exact(ti.haar_state(L, seed), L, s) for seed in range(4)]
    pur = [en.purity_exact(ti.haar_state(L, seed), L, s) for seed in range(4)]
    assert np.mean(vals) == pytest.approx(en.page_entropy(64, 256), abs=3e-3)
    assert np.mean(pur) == pytest.approx(en.haar_mean_purity(64, 256), rel=0.03)
    # Page: log2 d_S - d_S / (2 d_R ln 2) to leading order
    assert en.page_entropy(64, 256) == pytest.approx(6 - 64 / (2 * 256 * np.log(2)), abs=2e-3)


def test_lazy_matvec_is_the_reduced_density_matrix():
    L, s = 8, [6, 1, 3]
    psi = ti.haar_state(L, 5)
    M = en.psi_matrix(psi, L, s)
    X = probes.rademacher_probes(2, 3, 8, 0)
    rho = en.reduced_density_matrix(psi, L, s)
    assert np.allclose(en.rho_matvec(M, X), (rho @ X.T).T, rtol=1e-13, atol=1e-15)
    assert np.trace(rho).real == pytest.approx(1.0, abs=1e-13)


def test_purity_quadrature_is_exact_per_probe():
    # f = x^2 is a polynomial of degree 2 <= 2m - 1: each G_n is phi^dag rho^2 phi
    L, s = 10, [0, 1, 2, 3]
    psi = ti.haar_state(L, 7)
    r = en.slq_spectral_sum(psi, L, s, "purity", 5, 4, seed=11)
    rho = en.reduced_density_matrix(psi, L, s)
    X = probes.rademacher_probes(11, 5, 16, 0)
    want = np.array([np.vdot(x, rho @ (rho @ x)).real for x in X])
    assert np.allclose(r["G"], want, rtol=1e-12)


def test_slq_entropy_agrees_with_exact_within_its_error():
    L, s = 12, list(range(5))
    psi = ti.haar_state(L, 9)
    r = en.slq_spectral_sum(psi, L, s, "entropy", 32, 30, seed=1, reorth=True)
    ex = en.entropy_exact(psi, L, s)
    assert abs(r["value"] - ex) < 4 * r["value_se"] + 1e-3
    # operator on the smaller side: the complement of a 9-qubit S
    r2 = en.slq_spectral_sum(psi, L, list(range(3, 12)), "entropy", 32, 30, seed=1, reorth=True)
    assert r2["side"] == [0, 1, 2]
    ex2 = en.entropy_exact(psi, L, [0, 1, 2])
    assert abs(r2["value"] - ex2) < 4 * r2["value_se"] + 1e-3


def test_breakdown_gives_exact_entropy_of_low_rank_state():
    # Schmidt rank 2 across the cut: the Krylov space of rho_S is 2-dimensional
    # and every probe's quadrature is exact
    psi = ti.bell_pair_state(8, 2, 6)
    r = en.slq_spectral_sum(psi, 8, [0, 1, 2, 3], "entropy", 4, 6, seed=0)
    assert np.all(r["steps"] <= 2)
    X = probes.rademacher_probes(0, 4, 16, 0)
    rho = en.reduced_density_matrix(psi, 8, [0, 1, 2, 3])
    lam, V = scipy.linalg.eigh(rho)
    fvals = en.f_entropy(np.clip(lam, 0, None))
    want = [float(np.real(np.vdot(x, V @ (fvals * (V.conj().T @ x))))) for x in X]
    assert np.allclose(r["G"], want, rtol=1e-10, atol=1e-12)
