"""Pins for the oracle on sites of any local dimension (the method of Sec. V
for general d_A, d_B, d_C)."""
import numpy as np
import pytest
import scipy.linalg

import tnslq_inputs as ti
from oracle import exact, probes, slq


def test_two_level_sites_reduce_to_the_qubit_regrouping():
    L = 7
    psi = ti.haar_state(L, 3)
    for a, b in (([0, 4], [6, 1, 2]), ([5], [3]), ([2, 1, 0], [])):
        assert np.array_equal(exact.regroup_dims(psi, [2] * L, a, b), exact.regroup(psi, L, a, b))


@pytest.mark.parametrize("dims,i,j", [([3, 3, 2], 0, 1), ([2, 3, 4, 3], 3, 1), ([4, 2, 4], 2, 0)])
def test_maximally_entangled_pair_has_log2_d(dims, i, j):
    # Schmidt rank d with equal weights: |rho^{T_B}| has trace d, so E = log2 d
    psi = ti.max_entangled_pair_state_dims(dims, i, j)
    d = dims[i]
    P = exact.regroup_dims(psi, dims, [i], [j])
    assert exact.logneg_exact(P) == pytest.approx(np.log2(d), abs=1e-12)
    # both sites on one side: no entanglement across the cut
    others = [s for s in range(len(dims)) if s not in (i, j)]
    P = exact.regroup_dims(psi, dims, [i, j], others[:1])
    assert exact.logneg_exact(P) == pytest.approx(0.0, abs=1e-12)


def test_pure_state_schmidt_formula_for_qutrits():
    # empty environment: E = 2 log2 sum of the singular values of psi as d_A x d_B
    dims = [3, 3, 3, 2]
    psi = ti.haar_state_dims(dims, 5)
    a, b = [0, 3], [1, 2]
    P = exact.regroup_dims(psi, dims, a, b)
    M = np.asarray(psi).reshape(dims).transpose(a + b).reshape(6, 9)
    sv = np.linalg.svd(M, compute_uv=False)
    assert exact.logneg_exact(P) == pytest.approx(2 * np.log2(np.sum(sv)), abs=1e-12)


def test_partial_transpose_keeps_trace_and_hermiticity():
    dims = [3, 2, 4, 3]
    psi = ti.haar_state_dims(dims, 1)
    R = exact.rho_pt(exact.regroup_dims(psi, dims, [2], [0, 1]))
    assert np.trace(R).real == pytest.approx(1.0, abs=1e-13)
    assert np.allclose(R, R.conj().T, atol=1e-15)


def test_full_krylov_quadrature_is_exact_per_probe():
    # m = d_A d_B with reorthogonalisation: each G_n is phi^dagger |rho^{T_B}| phi
    dims = [3, 2, 3]
    psi = ti.haar_state_dims(dims, 2)
    P = exact.regroup_dims(psi, dims, [0], [2])
    R = exact.rho_pt(P)
    lam, V = scipy.linalg.eigh(R)
    absR = (V * np.abs(lam)) @ V.conj().T
    r = slq.slq_logneg_dims(psi, dims, [0], [2], 4, 9, seed=7, reorth=True)
    X = probes.rademacher_probes(7, 4, 9)
    want = np.array([np.vdot(x, absR @ x).real for x in X])
    assert np.allclose(r["G"], want, rtol=1e-10)
