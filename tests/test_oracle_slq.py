"""Pins for the oracle's SLQ (Sec. III, Algorithm 1; Sec. VIII) against
quadrature exactness, closed forms and the exact spectrum."""
import numpy as np
import pytest

import tnslq_inputs as ti
from oracle import exact, probes, slq


def _abs_op(R):
    w, v = np.linalg.eigh(R)
    return (v * np.abs(w)) @ v.conj().T


def _setup(L=8, a=(0, 1, 2), b=(4, 5), seed=1):
    psi = ti.haar_state(L, seed)
    P = exact.regroup(psi, L, list(a), list(b))
    return P, exact.rho_pt(P)


@pytest.mark.parametrize("power", [1, 2, 3])
def test_gauss_quadrature_exact_for_low_degree(power):
    # Gauss quadrature with m nodes integrates polynomials of degree <= 2m-1
    # exactly, so with m = 2: G = beta_1^2 F = phi^H X^p phi for p <= 3.
    P, R = _setup()
    phi = probes.rademacher_probes(4, 1, R.shape[0])[0]
    a, b, s = slq.lanczos(lambda v: R @ v, phi, 2)
    f = lambda x: x ** power  # noqa: E731
    G = b[0] ** 2 * slq.gauss_quadrature(a[:s], b[1:s], f)
    want = np.real(np.vdot(phi, np.linalg.matrix_power(R, power) @ phi))
    assert G == pytest.approx(want, rel=1e-12)


def test_full_krylov_gives_exact_bilinear_form():
    # m = dim with full reorthogonalisation: T_m is similar to X on the
    # Krylov space, so the quadrature of |x| is exact: G = phi^H |X| phi.
    P, R = _setup(L=7, a=(0, 1), b=(3, 5))
    absR = _abs_op(R)
    X = probes.rademacher_probes(8, 3, R.shape[0])
    out = slq.slq(lambda v: R @ v, X, m=R.shape[0], reorth=True)
    for k in range(3):
        want = np.real(np.vdot(X[k], absR @ X[k]))
        assert out["G"][k] == pytest.approx(want, rel=1e-9)


def test_bell_pair_every_probe_gives_two():
    # |rho^{T_B}| of a Bell pair in a |0> background is I/2 on the 4-dim Bell
    # block and 0 elsewhere: every unit-modulus probe gives G = 4/2 = 2, and
    # Lanczos breaks down after at most three steps (three distinct
    # eigenvalues: 1/2, -1/2, 0).
    L = 6
    psi = ti.bell_pair_state(L, 1, 4)
    out = slq.slq_logneg(psi, L, [0, 1], [3, 4], n_probes=6, n_steps=10, seed=2)
    assert np.allclose(out["G"], 2.0, atol=1e-12)
    assert np.all(out["steps"] <= 3)
    assert out["logneg"] == pytest.approx(1.0, abs=1e-12)
    # past the breakdown the trajectory repeats the exact value
    assert np.allclose(out["F"][:, 2:], out["F"][:, 2:3], atol=1e-15)


def test_basis_product_state_gives_one_per_probe():
    L = 6
    psi = ti.basis_product_state(L, [0, 1, 1, 0, 1, 0])
    out = slq.slq_logneg(psi, L, [0, 2], [3, 5], n_probes=4, n_steps=6, seed=0)
    assert np.allclose(out["G"], 1.0, atol=1e-12)
    assert out["logneg"] == pytest.approx(0.0, abs=1e-12)


def test_hutchinson_is_unbiased_and_variance_bounded():
    # Sec. VIII: per-probe variance bounded by the purity.  For {+-1, +-i}
    # probes Var(G) = sum_{i != j} |Y_ij|^2 with Y = |rho^{T_B}| (E z^2 = 0).
    P, R = _setup(L=8, a=(0, 1, 2), b=(4, 5), seed=3)
    Y = _abs_op(R)
    var_exact = float(np.sum(np.abs(Y) ** 2) - np.sum(np.abs(np.diag(Y)) ** 2))
    purity = float(np.real(np.trace(R @ R)))
    assert var_exact <= purity + 1e-15
    X = probes.rademacher_probes(21, 400, R.shape[0])
    out = slq.slq(lambda v: R @ v, X, m=R.shape[0] // 2, reorth=True)
    tn = exact.trace_norm_exact(P)
    assert abs(out["trace_norm"] - tn) < 4 * out["trace_norm_se"]
    s2 = np.var(out["G"], ddof=1)
    assert 0.7 * var_exact < s2 < 1.3 * var_exact


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_slq_matches_exact_small_haar(seed):
    # 10-qubit Haar state, A = 0-2, B = 3-5: 16 probes, 20 steps.
    psi = ti.haar_state(10, seed)
    P = exact.regroup(psi, 10, [0, 1, 2], [3, 4, 5])
    e = exact.logneg_exact(P)
    out = slq.slq_logneg(psi, 10, [0, 1, 2], [3, 4, 5], 16, 20, seed=seed)
    assert abs(out["logneg"] - e) < 4 * out["logneg_se"] + 0.01


def test_lazy_and_explicit_matvec_agree_inside_slq():
    psi = ti.haar_state(9, 8)
    r1 = slq.slq_logneg(psi, 9, [0, 1, 2], [5, 6], 3, 8, seed=1, matvec="explicit")
    r2 = slq.slq_logneg(psi, 9, [0, 1, 2], [5, 6], 3, 8, seed=1, matvec="lazy")
    assert np.allclose(r1["alpha"], r2["alpha"], rtol=0, atol=1e-14)
    assert np.allclose(r1["beta"], r2["beta"], rtol=0, atol=1e-14)


def test_ritz_values_lie_in_spectrum_range():
    P, R = _setup(L=8, a=(0, 1, 2), b=(3, 4, 5), seed=5)
    lam = np.linalg.eigvalsh(R)
    phi = probes.rademacher_probes(1, 1, R.shape[0])[0]
    a, b, s = slq.lanczos(lambda v: R @ v, phi, 12)
    T = np.diag(a[:s]) + np.diag(b[1:s], 1) + np.diag(b[1:s], -1)
    th = np.linalg.eigvalsh(T)
    assert th.min() >= lam.min() - 1e-12 and th.max() <= lam.max() + 1e-12


def test_hutchinson_stats_definitions():
    G = np.array([3.0, 5.0, 4.0, 8.0])
    st = slq.hutchinson_stats(G)
    assert st["trace_norm"] == 5.0
    assert st["trace_norm_se"] == pytest.approx(np.sqrt(np.sum((G - 5.0) ** 2) / 3) / 2)
    assert st["logneg"] == pytest.approx(np.log2(5.0))
    assert st["logneg_se"] == pytest.approx(st["trace_norm_se"] / (5.0 * np.log(2)))
    one = slq.hutchinson_stats(np.array([2.0]))
    assert one["logneg"] == 1.0 and np.isnan(one["logneg_se"])


def test_surrogate_features():
    from oracle import surrogate
    psi = ti.haar_state(10, 0)
    out = slq.slq_logneg(psi, 10, [0, 1, 2], [3, 4, 5], 16, 10, seed=0)
    f = surrogate.block_features(out["alpha"], out["beta"], 8, 8, 16)
    assert f.shape == (19,)
    # N alpha_1 = phi^H X phi averaged over probes, whose expectation is Tr X = 1
    assert abs(f[0] - 1.0) < 0.2
    assert list(f[16:]) == [3.0, 3.0, 4.0]
