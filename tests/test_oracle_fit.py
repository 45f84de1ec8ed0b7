"""Pins for the exponential-fit stopping rule of the oracle (Sec. III)."""
import numpy as np
import pytest
import scipy.optimize

import tnslq_inputs as ti
from oracle import exact, lanczos_fit as lf, probes, slq


@pytest.mark.parametrize("r", [0.85, 0.4, -0.3, -0.75, -0.95])
def test_noise_free_exponential_is_recovered_exactly(r):
    t = np.arange(8, dtype=float)
    y = 0.37 - 0.21 * r ** t
    f = lf.exponential_fit(y)
    assert f["f_inf"] == pytest.approx(0.37, abs=1e-12)
    assert f["r"] == pytest.approx(r, abs=1e-9)
    assert f["a"] == pytest.approx(-0.21, abs=1e-9)
    assert f["sigma"] < 1e-12


def test_constant_sequence_has_zero_uncertainty():
    f = lf.exponential_fit(np.full(6, 2.5))
    assert f["f_inf"] == pytest.approx(2.5, rel=1e-15)
    assert f["sigma"] < 1e-14


def _model(t, f_inf, a, r):
    return f_inf + a * r ** t


@pytest.mark.parametrize("seed,r_true", [(0, 0.6), (1, -0.7), (2, -0.4), (3, 0.8)])
def test_agrees_with_levenberg_marquardt(seed, r_true):
    # noisy data: the grid + bounded search and scipy's curve_fit (started from
    # several guesses, best residual kept) find the same optimum, and the
    # uncertainty matches curve_fit's sqrt(pcov[0, 0])
    rng = np.random.default_rng(seed)
    t = np.arange(8, dtype=float)
    y = 1.0 + 0.5 * r_true ** t + 1e-3 * rng.standard_normal(8)
    best = None
    for r0 in (-0.9, -0.5, -0.1, 0.1, 0.5, 0.9):
        try:
            p, cov = scipy.optimize.curve_fit(_model, t, y, p0=[y[-1], y[0] - y[-1], r0],
                                              bounds=([-np.inf, -np.inf, -0.99], [np.inf, np.inf, 0.99]))
        except RuntimeError:
            continue
        rss = float(np.sum((y - _model(t, *p)) ** 2))
        if best is None or rss < best[0]:
            best = (rss, p, cov)
    rss, p, cov = best
    f = lf.exponential_fit(y)
    assert f["rss"] <= rss * (1 + 1e-9)
    assert f["f_inf"] == pytest.approx(p[0], abs=1e-7)
    assert f["sigma"] == pytest.approx(np.sqrt(cov[0, 0]), rel=1e-3)


def test_sign_alternating_ratio_tracks_oscillating_convergence():
    # F_t = 1 + (-0.8)^t / (t + 1): geometric with a slowly varying amplitude,
    # the shape of |x| quadrature; the fit's limit is closer than the last value
    t = np.arange(8, dtype=float)
    y = 1.0 + (-0.8) ** (t + 6) / (t + 7)
    f = lf.exponential_fit(y)
    assert f["r"] < 0
    assert abs(f["f_inf"] - 1.0) < 0.2 * abs(y[-1] - 1.0)


def test_breakdown_makes_the_estimate_exact():
    # Bell pair between A and B in a product background: the Krylov space of
    # rho^T_B has dimension <= 3, every probe breaks down early and the
    # estimate is the exact quadrature value
    L = 4
    psi = ti.bell_pair_state(L, 0, 2)
    P = exact.regroup(psi, L, [0, 1], [2, 3])
    R = exact.rho_pt(P)
    X = probes.rademacher_probes(3, 4, 16, 0)
    r = slq.slq(lambda v: R @ v, X, 10)
    for n in range(4):
        s = lf.breakdown_step(r["alpha"][n], r["beta"][n])
        assert 0 < s <= 3
        est = lf.lanczos_estimate(r["F"][n], 10, s)
        assert est["sigma"] == 0.0 and est["f_inf"] == r["F"][n, s - 1]
    st = lf.fit_stats(r["F"], r["alpha"], r["beta"], 10)
    assert st["lanczos_err"] == 0.0
    assert st["trace_norm"] == pytest.approx(np.mean(r["G"]), rel=1e-14)


def test_fit_beats_the_last_quadrature_value_on_a_haar_state():
    # 14-qubit Haar state, A = 4-8, B = 9-13 (E = 4 qubits): the spectrum of
    # rho^T_B straddles 0, the quadrature of |x| converges with alternating
    # sign; at 10 steps the fitted limit is closer to the 40-step value than
    # F_10 for every probe, and the block error covers the true error
    L = 14
    psi = ti.haar_state(L, 1)
    a, b = list(range(4, 9)), list(range(9, 14))
    P = exact.regroup(psi, L, a, b)
    R = exact.rho_pt(P)
    X = probes.rademacher_probes(5, 6, 1024, 0)
    r = slq.slq(lambda v: R @ v, X, 40)
    for n in range(6):
        est = lf.lanczos_estimate(r["F"][n], 10, 0)
        ref = r["F"][n, -1]
        assert abs(est["f_inf"] - ref) < abs(r["F"][n, 9] - ref)
    st = lf.fit_stats(r["F"], r["alpha"], r["beta"], 10)
    assert abs(st["logneg"] - r["logneg"]) < 3 * st["logneg_err"]


def test_stop_step_meets_its_target_against_the_long_run():
    L = 14
    psi = ti.haar_state(L, 2)
    a, b = list(range(4, 9)), list(range(9, 14))
    P = exact.regroup(psi, L, a, b)
    R = exact.rho_pt(P)
    X = probes.rademacher_probes(7, 8, 1024, 0)
    r = slq.slq(lambda v: R @ v, X, 40)
    k = lf.fit_stop_step(r["F"], r["alpha"], r["beta"], 0.01)
    assert lf.FIT_MIN_POINTS + 1 <= k < 40
    st = lf.fit_stats(r["F"], r["alpha"], r["beta"], k)
    assert abs(st["logneg"] - r["logneg"]) <= 0.01 * max(abs(r["logneg"]), 1.0)
    # the step before did not meet the target
    if k > lf.FIT_MIN_POINTS + 1:
        prev = lf.fit_stats(r["F"], r["alpha"], r["beta"], k - 1)
        assert prev["logneg_err"] > 0.01 * max(abs(prev["logneg"]), 1.0)


def test_window_leaves_out_the_one_node_rule():
    # F_1 is never fitted: changing it changes no estimate
    rng = np.random.default_rng(4)
    F = 1.0 + (-0.7) ** np.arange(12) * 0.3 + 1e-4 * rng.standard_normal(12)
    G = F.copy()
    G[0] = 123.0
    for k in (6, 7, 9, 12):
        assert lf.lanczos_estimate(F, k)["f_inf"] == lf.lanczos_estimate(G, k)["f_inf"]
    # the window is F_2..F_k up to 8 points, then the last 8
    assert lf.lanczos_estimate(F, 9)["f_inf"] == lf.exponential_fit(F[1:9])["f_inf"]
    assert lf.lanczos_estimate(F, 12)["f_inf"] == lf.exponential_fit(F[4:12])["f_inf"]
    with pytest.raises(ValueError):
        lf.lanczos_estimate(F, 5)


def test_too_few_points_is_an_error():
    with pytest.raises(ValueError):
        lf.exponential_fit(np.ones(4))


# ------------------------------------------------------------ loop over probes
def _blocks(psi, L, a, b, K, m, seed):
    P = exact.regroup(psi, L, a, b)
    R = exact.rho_pt(P)
    n = P.shape[0] * P.shape[1]
    cache = {}

    def block(bi):
        if bi not in cache:
            X = probes.rademacher_probes(seed, K, n, bi * K)
            o = slq.slq(lambda v: R @ v, X, m)
            cache[bi] = (o["F"], o["alpha"], o["beta"])
        return cache[bi]
    return block, exact.logneg_exact(P)


def test_combined_error_is_the_standard_error_of_the_mean():
    import scipy.stats
    rng = np.random.default_rng(4)
    G = 3.0 + 0.2 * rng.standard_normal(24)
    c = lf.combined_stats(G, np.zeros(24))
    assert c["trace_norm_se"] == pytest.approx(float(scipy.stats.sem(G)), rel=1e-12)
    assert c["logneg"] == pytest.approx(np.log2(np.mean(G)), rel=1e-14)
    # with a Lanczos part the errors add in quadrature
    c2 = lf.combined_stats(G, np.full(24, 0.05))
    assert c2["logneg_err"] == pytest.approx(np.hypot(scipy.stats.sem(G), 0.05) / (np.mean(G) * np.log(2.0)),
                                             rel=1e-12)
    # one probe: the Hutchinson error is unknown, never converged
    assert lf.combined_stats(G[:1], np.zeros(1))["logneg_err"] == np.inf


def test_block_lanczos_stop_comes_no_later_than_the_combined_rule():
    L, a, b = 14, list(range(4, 9)), list(range(9, 14))
    block, _ = _blocks(ti.haar_state(L, 2), L, a, b, 4, 30, 7)
    F, al, be = block(0)
    assert lf.block_lanczos_stop_step(F, al, be, 0.01) <= lf.fit_stop_step(F, al, be, 0.01)


def test_probe_loop_stops_at_the_first_block_count_meeting_the_target():
    # blocks of 8 probes (the first Hutchinson check sees 8 samples): this
    # state needs two; replaying every prefix of blocks by brute force finds
    # the same count
    L, a, b = 12, [0, 1, 2, 3], [6, 7, 8, 9]
    block, e_exact = _blocks(ti.haar_state(L, 1), L, a, b, 8, 30, 3)
    tol = 0.01
    r = lf.probe_loop(block, 8, 256, tol)
    G, S, first = [], [], None
    for bi in range(32):
        F, al, be = block(bi)
        st = lf.fit_stats(F, al, be, lf.block_lanczos_stop_step(F, al, be, tol))
        G.extend(st["G"])
        S.extend(st["sigma"])
        c = lf.combined_stats(np.array(G), np.array(S))
        if c["logneg_err"] <= tol * max(abs(c["logneg"]), 1.0):
            first = bi + 1
            break
    assert first is not None and r["n_probes_used"] == 8 * first > 8
    assert r["logneg"] == pytest.approx(lf.combined_stats(np.array(G), np.array(S))["logneg"], rel=1e-14)
    # and the estimate is within its stated error of the exact value
    assert abs(r["logneg"] - e_exact) <= 3 * r["logneg_err"]


def test_probe_loop_respects_the_probe_budget():
    L, a, b = 12, [0, 1, 2, 3], [6, 7, 8, 9]
    block, _ = _blocks(ti.haar_state(L, 1), L, a, b, 4, 24, 3)
    r = lf.probe_loop(block, 4, 11, 1e-6)   # unreachable target: 2 blocks fit in 11 probes
    assert r["n_probes_used"] == 8 and len(r["stops"]) == 2
    assert r["logneg_err"] > 1e-6


# ------------------------------------------------------------ model term
@pytest.mark.parametrize("j_end,n", [(6, 5), (9, 8), (17, 8)])
def test_algebraic_law_is_recovered_exactly(j_end, n):
    # noise-free F_j = 0.81 + 0.37 (-1)^j / j^2 - 0.05 / j^2 over steps
    # j_end - n + 1 .. j_end: the algebraic fit returns the limit
    j = np.arange(j_end - n + 1, j_end + 1, dtype=float)
    y = 0.81 + 0.37 * (-1.0) ** j / j ** 2 - 0.05 / j ** 2
    assert lf.algebraic_fit(y, j_end) == pytest.approx(0.81, abs=1e-13)


def test_model_term_is_the_distance_between_the_two_limits():
    # on an algebraic trajectory the model term is exactly how far the
    # exponential's limit lies from the true one; a constant trajectory has
    # no model error and no fit error
    j = np.arange(1, 13, dtype=float)
    F = 0.5 + 0.3 * (-1.0) ** j / j ** 2 + 0.02 / j ** 2
    for k in (6, 9, 12):
        est = lf.lanczos_estimate(F, k)
        assert est["model"] == pytest.approx(abs(est["f_inf"] - 0.5), abs=1e-13)
        assert est["sigma"] == pytest.approx(np.hypot(est["sigma_fit"], est["model"]), rel=1e-15)
        assert est["sigma"] >= abs(est["f_inf"] - 0.5)
    c = lf.lanczos_estimate(np.full(10, 0.25), 10)
    assert c["f_inf"] == pytest.approx(0.25, rel=1e-15) and c["sigma"] < 1e-14


def _coverage_cases():
    # 21 Haar states of 12-14 qubits with small environments (d_E = 4-16, the
    # regime of the 26-qubit rho_AB: the spectrum straddles 0) and three cuts
    out = []
    for L, a, b in ((12, list(range(2, 7)), list(range(7, 12))), (13, list(range(3, 8)), list(range(8, 13))),
                    (14, list(range(0, 4)), list(range(4, 10)))):
        for s in range(7):
            out.append((L, a, b, 40 + 7 * L + s))
    return out


def test_stated_lanczos_error_covers_the_long_run():
    # at the fit rule's +-1% stop, the stated Lanczos error (in bits) must
    # cover the distance to the converged value on the same probes on at least
    # 68% of the states (a one-sigma bar); the converged value is the mean of
    # the plain quadrature estimates over steps 71-80, which averages the last
    # alternation of the quadrature
    cover, steps = [], []
    for L, a, b, seed in _coverage_cases():
        P = exact.regroup(ti.haar_state(L, seed), L, a, b)
        R = exact.rho_pt(P)
        X = probes.rademacher_probes(seed, 8, R.shape[0], 0)
        r = slq.slq(lambda v: R @ v, X, 80)
        e_long = np.mean([np.log2(np.mean(r["beta"][:, 0] ** 2 * r["F"][:, j])) for j in range(70, 80)])
        k = lf.fit_stop_step(r["F"], r["alpha"], r["beta"], 0.01)
        st = lf.fit_stats(r["F"], r["alpha"], r["beta"], k)
        stated = st["lanczos_err"] / (st["trace_norm"] * np.log(2.0))
        cover.append(abs(st["logneg"] - e_long) <= stated)
        steps.append(k)
    assert len(cover) >= 20
    assert np.mean(cover) >= 0.68, (np.mean(cover), steps)
    assert max(steps) < 20        # and the rule still stops early


def test_unmet_target_reports_the_plain_estimate_of_the_last_step():
    # a 12-qubit brickwork state of depth 3 does not meet a 1e-6 target in
    # 20 steps: the run reports what plain SLQ of 20 steps gives (the
    # oracle's SLQ, pinned against exact spectra elsewhere), with the fit's
    # Lanczos error; a 1% target on a Haar state is met and reports the fit
    L, a, b = 12, list(range(1, 6)), list(range(6, 11))
    psi = ti.brickwork_state(L, 3, 0)
    r = slq.slq_logneg(psi, L, a, b, 8, 20, seed=2)
    out = lf.fit_rule_result(r["F"], r["alpha"], r["beta"], 1e-6)
    assert not out["met"] and out["step"] == 20
    assert out["logneg"] == pytest.approx(r["logneg"], abs=1e-12)
    st = lf.fit_stats(r["F"], r["alpha"], r["beta"], 20)
    assert out["lanczos_err"] == pytest.approx(st["lanczos_err"] / (st["trace_norm"] * np.log(2.0)), rel=1e-12)
    assert out["lanczos_err"] > 1e-6 * max(abs(out["logneg"]), 1.0)
    psi = ti.haar_state(L, 4)
    r = slq.slq_logneg(psi, L, a, b, 8, 20, seed=2)
    out = lf.fit_rule_result(r["F"], r["alpha"], r["beta"], 0.01)
    k = lf.fit_stop_step(r["F"], r["alpha"], r["beta"], 0.01)
    assert out["met"] and out["step"] == k < 20
    assert out["logneg"] == lf.fit_stats(r["F"], r["alpha"], r["beta"], k)["logneg"]
