"""The package's host-side arithmetic outside the run-time path (the
surrogate's training features and early-estimate labels, and the replay of the
step-difference rule in the experiment drivers) against the oracle's
definitions, on trajectories from the oracle's SLQ."""
import numpy as np
import pytest

import tnslq_inputs as ti
from oracle import slq, step_difference, surrogate as osur
from paper_1809_01685_amd import experiments
from paper_1809_01685_amd import surrogate as psur


@pytest.fixture(scope="module")
def runs():
    out = []
    for L, a, b, seed in ((10, [0, 1, 2], [3, 4, 5], 0), (9, [1, 2], [5, 6, 7], 3), (8, [0, 1, 2], [3, 4], 5)):
        psi = ti.haar_state(L, seed)
        r = slq.slq_logneg(psi, L, a, b, 8, 24, seed=seed + 1)
        r["steps_done"] = 24
        r["dims"] = (1 << len(a), 1 << len(b), 1 << (L - len(a) - len(b)))
        out.append(r)
    return out


def test_training_features_and_labels_match_the_oracle(runs):
    for r in runs:
        d_a, d_b, d_e = r["dims"]
        for n_early in (4, 5, 8):
            f = psur.features_from_coefficients(r["alpha"], r["beta"], d_a, d_b, d_e, n_early)
            assert np.allclose(f, osur.block_features(r["alpha"], r["beta"], d_a, d_b, d_e, n_early), rtol=1e-15,
                               atol=0)
        for j in (6, 8, 24):
            assert psur.estimate_at(r["beta"], r["F"], j) == pytest.approx(
                step_difference.block_estimate(r["beta"], r["F"], j)["logneg"], abs=1e-14)


@pytest.mark.parametrize("tol", [0.05, 0.01, 0.002])
def test_replayed_difference_rule_matches_the_oracle(runs, tol):
    for r in runs:
        E, dE = experiments._trajectory(r)
        assert experiments._adaptive_stop(E, dE, tol) == step_difference.stop_step(r["beta"], r["F"], tol)
