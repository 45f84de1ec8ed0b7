"""Pins for the oracle's early-stopping decisions: the learned stop's
features, input map and head (oracle.surrogate) and the step-difference rule
(oracle.step_difference), against closed forms and independent routines."""
import math

import numpy as np
import pytest
import scipy.stats

import tnslq_inputs as ti
from oracle import mlp, probes, slq, step_difference, surrogate


# ---------------------------------------------------------------- features
def test_features_of_a_jacobi_matrix_are_its_entries():
    # Lanczos started from e_1 on a Jacobi matrix (real symmetric tridiagonal,
    # positive off-diagonal) reproduces that matrix: its alpha_k is the k-th
    # diagonal entry and beta_{k+1} the k-th off-diagonal one.  So the
    # features are d_A d_B times the first eight entries of each, which puts
    # every alpha and beta index in its place.
    n = 16
    diag = 0.05 * np.arange(1, n + 1) - 0.3
    off = 1.0 / np.arange(2, n + 1)
    T = np.diag(diag) + np.diag(off, 1) + np.diag(off, -1)
    e1 = np.zeros(n, dtype=np.complex128)
    e1[0] = 1.0
    a, b, s = slq.lanczos(lambda v: T @ v, e1, 10, reorth=True)
    assert s == 10 and b[0] == 1.0
    f = surrogate.block_features(a[None, :], b[None, :], 4, 4, 2)
    assert np.allclose(f[:8], n * diag[:8], rtol=0, atol=1e-12)
    assert np.allclose(f[8:16], n * off[:8], rtol=0, atol=1e-12)
    assert list(f[16:]) == [2.0, 2.0, 1.0]
    # a network trained on fewer early steps reads them in the same slots,
    # the later slots of each kind left zero
    f5 = surrogate.block_features(a[None, :], b[None, :], 4, 4, 2, n_early=5)
    assert np.allclose(f5[:5], n * diag[:5], rtol=0, atol=1e-12) and not f5[5:8].any()
    assert np.allclose(f5[8:13], n * off[:5], rtol=0, atol=1e-12) and not f5[13:16].any()
    assert list(f5[16:]) == [2.0, 2.0, 1.0]


def test_features_of_a_bell_pair_in_closed_form():
    # A Bell pair with A and B one qubit each: rho^{T_B} = SWAP / 2
    # (eigenvalues +1/2 three times, -1/2 once).  For a probe phi of four
    # unit-modulus entries, with c = Re(conj(phi_01) phi_10):
    #   alpha_1 = phi^H SWAP phi / 8 = (1 + c) / 4,
    #   beta_2 = sqrt(1/4 - alpha_1^2), and when beta_2 > 0 the Krylov space
    #   is two-dimensional with eigenvalues +-1/2, so alpha_2 = -alpha_1 and
    #   the recurrence stops (beta_3 = 0, later coefficients 0).
    L, K = 6, 16
    psi = ti.bell_pair_state(L, 1, 4)
    out = slq.slq_logneg(psi, L, [1], [4], K, 10, seed=3)
    X = probes.rademacher_probes(3, K, 4)
    c = np.real(np.conj(X[:, 1]) * X[:, 2])
    a1 = (1.0 + c) / 4.0
    b2 = np.sqrt(0.25 - a1 * a1)
    a2 = np.where(b2 > 0, -a1, 0.0)
    want = np.zeros(19)
    want[0] = 4.0 * a1.mean()
    want[1] = 4.0 * a2.mean()
    want[8] = 4.0 * b2.mean()
    want[16:] = [1.0, 1.0, 4.0]
    f = surrogate.block_features(out["alpha"], out["beta"], 2, 2, 16)
    assert np.allclose(f, want, rtol=0, atol=1e-12)
    assert len(set(np.round(c, 6))) > 1   # the probes cover several cases


# ---------------------------------------------------------------- input map
def test_network_input_map_on_a_pass_through_network():
    # A network whose only path is input i -> unit 0 -> unit 0 -> u0 with
    # weights 1 (exact in BF16) and zero biases outputs relu(xhat_i).
    # Feature 3 = sinh(3) maps to asinh = 3; with mean 1 and scale 0.5 the
    # standardised value is 4.  Feature 17 (log2 d_B, not mapped) = 5 with
    # mean 2 and scale 1.5 gives 2.
    for i, x_i, mean, scale, want in ((3, math.sinh(3.0), 1.0, 0.5, 4.0), (17, 5.0, 2.0, 1.5, 2.0)):
        theta = np.zeros(mlp.N_PARAMS)
        p = mlp.unpack(theta)
        p["W1"][0, i] = 1.0
        p["W2"][0, 0] = 1.0
        p["W3"][0, 0] = 1.0
        theta = mlp.pack(p)
        norm = np.concatenate([np.zeros(19), np.ones(19)])
        norm[i], norm[19 + i] = mean, scale
        x = np.zeros(19)
        x[i] = x_i
        u, _ = mlp.forward(theta, surrogate.network_input(x, norm)[None, :])
        assert u[0, 0] == pytest.approx(want, rel=1e-6)
        assert u[0, 1] == 0.0


# ---------------------------------------------------------------- head
def _bias_only_network(u0, u1):
    theta = np.zeros(mlp.N_PARAMS)
    theta[-2:] = [u0, u1]
    return theta


def test_early_estimate_is_the_eight_step_slq_estimate():
    # E_early from 20-step trajectories equals the estimate of an SLQ run
    # stopped after 8 steps on the same probes (a separate oracle path).
    psi = ti.haar_state(10, 4)
    a, b = [0, 1, 2], [3, 4, 5]
    long = slq.slq_logneg(psi, 10, a, b, 8, 20, seed=5)
    short = slq.slq_logneg(psi, 10, a, b, 8, 8, seed=5)
    d = surrogate.decision(_bias_only_network(0.0, 0.0), np.concatenate([np.zeros(19), np.ones(19)]), 1.0,
                           long["alpha"], long["beta"], long["F"], 8, 8, 16, tol=0.01)
    assert d["e_early"] == pytest.approx(short["logneg"], abs=1e-13)
    assert abs(d["e_early"] - long["logneg"]) > 1e-6   # step 8 differs from step 20 here


def test_head_and_accept_rule_on_a_bell_pair():
    # Every probe of a Bell pair gives G = 2, so E_early = 1 exactly; a
    # network with zero weights outputs its last bias (u0, u1).  Then
    # mu = 1 + y u0 and sigma = y exp(u1 / 2), and the early result is
    # accepted exactly when sigma <= tol max(|mu|, 1).
    L = 6
    psi = ti.bell_pair_state(L, 1, 4)
    out = slq.slq_logneg(psi, L, [0, 1], [3, 4], 8, 10, seed=2)
    y, u0, u1 = 0.25, 2.0, math.log(0.04)     # y is exact in FP32
    norm = np.concatenate([np.zeros(19), np.ones(19)])
    theta = _bias_only_network(u0, u1)
    d = surrogate.decision(theta, norm, y, out["alpha"], out["beta"], out["F"], 4, 4, 16, tol=0.01)
    assert d["e_early"] == pytest.approx(1.0, abs=1e-14)
    assert d["mu"] == pytest.approx(1.5, abs=1e-14)
    assert d["sigma"] == pytest.approx(0.05, rel=1e-12)
    # threshold tol * 1.5: accepted above sigma / 1.5, refused below
    for tol, acc in ((0.05 / 1.5 * 1.001, True), (0.05 / 1.5 * 0.999, False), (1.0, True), (1e-3, False)):
        assert surrogate.decision(theta, norm, y, out["alpha"], out["beta"], out["F"], 4, 4, 16,
                                  tol=tol)["accept"] is acc
    # a negative mu: max(|mu|, 1) uses |mu| = 3
    d = surrogate.decision(_bias_only_network(-16.0, u1), norm, y, out["alpha"], out["beta"], out["F"], 4, 4, 16,
                           tol=0.05 / 3.0 * 1.001)
    assert d["mu"] == pytest.approx(-3.0, abs=1e-14) and d["accept"]
    # a non-finite network output is never accepted
    d = surrogate.decision(_bias_only_network(0.0, np.inf), norm, y, out["alpha"], out["beta"], out["F"], 4, 4, 16,
                           tol=1e9)
    assert not d["accept"]


# ---------------------------------------------------------------- step-difference rule
def test_difference_rule_stops_at_six_when_converged():
    # Bell pair and computational-basis product state: once every probe has
    # broken down (step s at most 3) its quadrature is exact, G = 2 (Bell) or
    # G = 1 (product) per probe, so the error on the mean is 0 and E_j -
    # E_{j-5} = 0 from j = s + 5 on.  For the product state rho^{T_B} is a
    # rank-one projector and even the one-node rule is exact (|x| = x on it),
    # so the rule stops at its first step, 6.
    L = 6
    for psi, a, b, e in ((ti.bell_pair_state(L, 1, 4), [0, 1], [3, 4], 1.0),
                         (ti.basis_product_state(L, [0, 1, 1, 0, 1, 0]), [0, 1], [3, 4], 0.0)):
        out = slq.slq_logneg(psi, L, a, b, 8, 12, seed=1)
        r = step_difference.run(out["beta"], out["F"], tol=1e-9)
        want = 6 if e == 0.0 else 5 + int(out["steps"].max())
        assert 1 < out["steps"].max() <= 3 or e == 0.0
        assert r["steps"] == want
        assert r["logneg"] == pytest.approx(e, abs=1e-13)
        assert r["lanczos_err"] == pytest.approx(0.0, abs=1e-13)


def test_difference_rule_on_geometric_trajectories():
    # F_j,n = c_n (1 + r^j): T_j = mean(c) (1 + r^j), so the relative error on
    # the mean is sem(c) / mean(c) at every step (scipy's standard error) and
    # E_j - E_{j-5} = log2((1 + r^j) / (1 + r^(j-5))).  The rule stops at the
    # first j >= 6 where the root sum of squares of the two meets the target.
    rng = np.random.default_rng(7)
    K, m = 12, 40
    c = 1.0 + 0.01 * rng.standard_normal(K)
    for r_ in (0.5, -0.6, 0.8):
        j = np.arange(1, m + 1)
        F = c[:, None] * (1.0 + r_ ** j)[None, :]
        beta = np.zeros((K, m + 1))
        beta[:, 0] = 1.0
        dE = scipy.stats.sem(c) / np.mean(c) / math.log(2.0)
        tol = 0.004
        want = m
        for jj in range(6, m + 1):
            e = math.log2(np.mean(c) * (1 + r_ ** jj))
            dl = math.log2((1 + r_ ** jj) / (1 + r_ ** (jj - 5)))
            if math.hypot(dE, dl) <= tol * max(abs(e), 1.0):
                want = jj
                break
        assert 6 < want < m
        got = step_difference.run(beta, F, tol)
        assert got["steps"] == want
        assert got["logneg_se"] == pytest.approx(dE, rel=1e-10)
        # a looser target never stops later, a tighter one never earlier
        assert step_difference.stop_step(beta, F, 2 * tol) <= want <= step_difference.stop_step(beta, F, tol / 2)


def test_difference_rule_single_probe_and_no_stop():
    # One probe: the error on the mean is undefined and counts as 0, so the
    # rule tests the step difference alone; a target nothing meets runs to
    # the last step.
    m = 30
    j = np.arange(1, m + 1)
    F = (2.0 + 0.5 ** j)[None, :]
    beta = np.ones((1, m + 1))
    got = step_difference.run(beta, F, tol=1e-3)
    k = next(jj for jj in range(6, m + 1)
             if abs(math.log2((2 + 0.5 ** jj) / (2 + 0.5 ** (jj - 5)))) <= 1e-3 * math.log2(2 + 0.5 ** jj))
    assert got["steps"] == k and np.isnan(got["logneg_se"])
    assert step_difference.run(beta, F, tol=1e-30)["steps"] == m
