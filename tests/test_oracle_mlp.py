"""Pins for the surrogate network's FP64 reference."""
import numpy as np
import pytest

import tnslq_inputs as ti
from oracle import mlp


def _batch(seed=1, B=16):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((B, mlp.N_IN)), rng.standard_normal(B)


def test_parameter_count():
    assert mlp.N_PARAMS == 71426
    assert ti.mlp_init_params(0).size == mlp.N_PARAMS


def test_gradient_matches_finite_differences():
    th = ti.mlp_init_params(0).astype(np.float64)
    x, r = _batch()
    _, g, _ = mlp.loss_and_grad(th, x, r, quantise=False)
    rng = np.random.default_rng(2)
    idx = np.concatenate([rng.integers(0, mlp.N_PARAMS, 40), [71424, 71425, 4864, 5119]])
    eps = 1e-6
    for i in idx:
        tp, tm = th.copy(), th.copy()
        tp[i] += eps
        tm[i] -= eps
        fd = (mlp.loss_and_grad(tp, x, r, False)[0] - mlp.loss_and_grad(tm, x, r, False)[0]) / (2 * eps)
        assert g[i] == pytest.approx(fd, rel=1e-5, abs=1e-9)


def test_quantised_gradient_is_straight_through():
    th = ti.mlp_init_params(3).astype(np.float64)
    x, r = _batch(4)
    p = mlp.unpack(th)
    for k in ("W1", "W2", "W3"):
        p[k] = mlp.bf16_round(p[k])
    thq = mlp.pack(p)
    lq, gq, _ = mlp.loss_and_grad(th, x, r, quantise=True)
    l2, g2, _ = mlp.loss_and_grad(thq, x, r, quantise=False)
    assert lq == l2 and np.array_equal(gq, g2)


def test_bf16_rounding_ties_to_even():
    one = 1.0
    assert mlp.bf16_round(np.array([one]))[0] == 1.0
    assert mlp.bf16_round(np.array([1 + 2.0 ** -8]))[0] == 1.0             # tie -> even (down)
    assert mlp.bf16_round(np.array([1 + 3 * 2.0 ** -8]))[0] == 1 + 2.0 ** -6  # tie -> even (up)
    assert mlp.bf16_round(np.array([1 + 2.0 ** -8 + 2.0 ** -20]))[0] == 1 + 2.0 ** -7
    assert mlp.bf16_round(np.array([-3.0]))[0] == -3.0


def test_bf16_rounding_agrees_with_torch():
    torch = pytest.importorskip("torch")
    x = np.random.default_rng(0).standard_normal(100000).astype(np.float32) * 7
    want = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(mlp.bf16_round(x), want)


def test_adam_first_step_closed_form():
    # t = 1: mhat = g, vhat = g^2, so the update is lr * g / (|g| + eps)
    rng = np.random.default_rng(0)
    th = rng.standard_normal(50)
    g = rng.standard_normal(50)
    z = np.zeros(50)
    th1, m, v = mlp.adam_step(th, z, z, g, 1, lr=1e-3)
    assert np.allclose(th - th1, 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_nll_gradient_at_optimum_is_zero_for_mean():
    # the mean output's gradient vanishes when it equals the target
    th = ti.mlp_init_params(5).astype(np.float64)
    x, _ = _batch(6, 8)
    u, _ = mlp.forward(th, x)
    _, g, _ = mlp.loss_and_grad(th, x, u[:, 0])
    # with d = 0 the log-variance gradient is 0.5/B per sample and the mean's is 0;
    # b3[0]'s gradient is the sum of mean-gradients
    assert abs(g[-2]) < 1e-15
    assert g[-1] == pytest.approx(0.5, rel=1e-12)


def test_input_transform_compresses_only_the_lanczos_features():
    rng = np.random.default_rng(3)
    y = rng.uniform(-15, 15, size=(5, 19))
    x = y.copy()
    x[:, :16] = np.sinh(y[:, :16])            # values spanning ~1e-6 .. 1e6
    t = mlp.input_transform(x)
    assert np.allclose(t[:, :16], y[:, :16], rtol=1e-12, atol=1e-12)
    assert np.array_equal(t[:, 16:], x[:, 16:])
    assert np.allclose(mlp.standardise(x, 1.0, 2.0), (t - 1.0) / 2.0)
