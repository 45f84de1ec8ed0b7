"""The learned early stop: what the trained network gains over the method
without it, and that its run-time entry point (features, network, head and
accept rule after the network's early Lanczos steps) matches the oracle's
decision.

Gain is measured against full SLQ (40 steps, 32 probes) as the reference, on
instances the network never saw:
  * the held-out 10% of the method-generated training set (split by instance);
  * freshly drawn instances from the same family with new seeds.
The comparison baseline is the same early SLQ estimate without the network.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu
T = pytest.importorskip("paper_1809_01685_amd")
from paper_1809_01685_amd import surrogate as S  # noqa: E402


@pytest.fixture(scope="module")
def model():
    return S.Model.load()


def _gain(mu, sigma, e8, ef):
    err_m, err_8 = np.abs(mu - ef), np.abs(e8 - ef)
    tol = 0.01 * np.maximum(np.abs(ef), 1.0)
    acc = sigma <= 0.01 * np.maximum(np.abs(mu), 1.0)
    return err_m, err_8, tol, acc


def test_network_beats_early_slq_on_held_out_split(dev, model):
    with np.load(S.os.path.join(S.WEIGHTS_DIR, "train_set.npz")) as f:
        data = {k: f[k] for k in f.files}
    X, e_early = S.dataset_features(data, model.feature_steps)
    ef = data["e_full"]
    va = np.array(model.meta["val_index"])
    mu, sigma = S.predict(model, X[va], e_early[va], dev)
    err_m, err_8, tol, acc = _gain(mu, sigma, e_early[va], ef[va])
    print(f"held-out split: MAE {err_m.mean():.4f} vs {err_8.mean():.4f}, median {np.median(err_m):.5f} vs "
          f"{np.median(err_8):.5f}, accepted {acc.mean():.3f}, accepted within 1%: {np.mean(err_m[acc] <= tol[acc]):.3f}")
    assert err_m.mean() < err_8.mean()
    assert np.median(err_m) < np.median(err_8)
    # the stop is taken mostly when it is safe
    assert acc.mean() > 0.3
    assert np.mean(err_m[acc] <= tol[acc]) >= 0.95


def test_network_gain_on_fresh_instances(dev, model):
    rng = np.random.default_rng(2024)
    n_early = model.feature_steps
    rows = []
    for _ in range(100):
        inst = S.draw_instance(rng, 16, 20)
        out = S.run_instance(inst, dev, seed=inst.seed + 1)
        rows.append((S.features(out["A"], out["B"], *out["dims"], n_early), out["E"][n_early - 1], out["e_full"]))
    X = np.array([r[0] for r in rows])
    e8 = np.array([r[1] for r in rows])
    ef = np.array([r[2] for r in rows])
    mu, sigma = S.predict(model, X, e8, dev)
    err_m, err_8, tol, acc = _gain(mu, sigma, e8, ef)
    print(f"fresh: MAE {err_m.mean():.4f} vs {err_8.mean():.4f}, median {np.median(err_m):.5f} vs "
          f"{np.median(err_8):.5f}, accepted {acc.mean():.3f}")
    # mean error improves; the median is reported (at this sample size it is
    # dominated by the many instances the early estimate already gets right)
    assert err_m.mean() < err_8.mean()
    assert acc.sum() >= 10 and np.mean(err_m[acc] <= tol[acc]) >= 0.9


def test_learned_stop_beats_the_fit_rule_on_fresh_haar_states(dev, model):
    # Haar states the network never saw (new seeds, 20-22 qubits, contiguous
    # A and B), 8 probes as at the 26-qubit workload: the learned stop is
    # taken earlier than the exponential-fit stop at the same +-1% target,
    # and on average lands at least as close to 40-step SLQ on the same probes
    import torch
    import tnslq_inputs as ti
    rng = np.random.default_rng(77)
    rows = []
    for i in range(8):
        L = int(rng.integers(20, 23))
        a, b = ti.random_contiguous_partition(L, rng)
        psi = ti.haar_state_torch(L, 1000 + i, dev, torch.complex64)
        ref = T.tnslq_logneg(psi, L, a, b, 8, 40, precision="bf16x3", seed=i, want_arrays=False)["logneg"]
        fit = T.tnslq_logneg(psi, L, a, b, 8, 40, precision="bf16x3", seed=i, stop_tol=0.01, stop_rule="fit",
                             want_arrays=False)
        s = S.surrogate_logneg(model, psi, L, a, b, 8, 40, tol=0.01, precision="bf16x3", seed=i, stop_tol=0.01,
                               stop_rule="fit")
        rows.append((fit["steps_done"], s["steps_done"], not s["used_fallback"], abs(fit["logneg"] - ref),
                     abs(s["logneg"] - ref), 0.01 * max(abs(ref), 1.0)))
        print(f"L={L} |A|={len(a)} |B|={len(b)}: fit rule {fit['steps_done']} steps err {rows[-1][3]:.4f}, "
              f"learned stop {s['steps_done']} steps err {rows[-1][4]:.4f}, accepted {rows[-1][2]}")
    r = np.array(rows, dtype=float)
    assert r[:, 2].all()                       # every Haar case stops early
    assert (r[:, 1] < r[:, 0]).all()           # before the fit rule's stop
    assert (r[:, 4] <= r[:, 5]).all()          # within the +-1% target
    assert r[:, 4].mean() <= r[:, 3].mean()    # and no less accurate on average


def _decision_margin_ok(d, tol):
    # the accept decision compares sigma with tol max(|mu|, 1); both sides
    # compute it in double from FP32 network outputs, so only a margin below
    # the network's rounding leaves the flag open
    thr = tol * max(abs(d["mu"]), 1.0)
    return abs(d["sigma"] - thr) > 1e-4 * thr


@pytest.mark.parametrize("tol", [0.01, 1e9, 1e-12])
def test_surrogate_entry_point_matches_oracle_decision(dev, model, tol):
    # the run-time path (the network's early FP64 Lanczos steps, the feature
    # kernel, the network, mu = E_early + y_scale u0, sigma = y_scale
    # exp(u1 / 2) and the accept rule) against the oracle's decision on the
    # oracle's own coefficients for the same probes
    import torch
    import tnslq_inputs as ti
    from oracle import exact, probes, slq, surrogate as osur
    L, a, b, K, m = 12, list(range(2, 7)), list(range(7, 12)), 16, 24
    psi = ti.haar_state(L, 5)
    r = S.surrogate_logneg(model, torch.from_numpy(psi).to(dev), L, a, b, K, m, tol=tol, precision="fp64", seed=3,
                           operator="lazy")
    R = exact.rho_pt(exact.regroup(psi, L, a, b))
    o = slq.slq(lambda v: R @ v, probes.rademacher_probes(3, K, 1 << 10), m)
    d = osur.decision(model.params, model.norm, model.y_scale, o["alpha"], o["beta"], o["F"], 1 << 5, 1 << 5,
                      1 << 2, tol, n_early=model.feature_steps)
    assert r["e_early"] == pytest.approx(d["e_early"], abs=1e-10)
    assert r["mu"] == pytest.approx(d["mu"], abs=1e-5 * max(1.0, abs(d["mu"])))
    assert r["sigma"] == pytest.approx(d["sigma"], rel=1e-5)
    if _decision_margin_ok(d, tol):
        assert r["used_fallback"] == (not d["accept"])
    if r["used_fallback"]:
        # the fallback is full SLQ: the oracle's estimate after m steps
        assert r["steps_done"] == m
        assert r["logneg"] == pytest.approx(o["logneg"], abs=1e-10 * max(1.0, abs(o["logneg"])))
    else:
        assert r["steps_done"] == model.feature_steps
        assert r["logneg"] == r["mu"] and r["logneg_se"] == r["sigma"]


def test_fallback_runs_full_slq(dev, model):
    import torch
    import tnslq_inputs as ti
    L, a, b = 16, [0, 1, 2, 3, 4], [8, 9, 10]
    psi = ti.brickwork_state_torch(L, 3, 9, dev, torch.complex64)
    full = T.tnslq_logneg(psi, L, a, b, 16, 24, precision="bf16x3", seed=1)
    r = S.surrogate_logneg(model, psi, L, a, b, 16, 24, tol=1e-12, precision="bf16x3", seed=1)
    assert r["used_fallback"] and r["steps_done"] == 24
    assert r["logneg"] == pytest.approx(full["logneg"], abs=1e-12)
    assert r["e_full"] == pytest.approx(full["logneg"], abs=1e-12)
