"""FP64 reference of the early-stopping surrogate network.

Oracle, test infrastructure only.  The paper has no learned component; this
is the project's addition: a 3-layer perceptron 19 -> 256 -> 256 -> 2 with
ReLU, weights used in BF16 (rounded to nearest even from FP32 master
weights), trained with a Gaussian negative log-likelihood and Adam
(Kingma & Ba 2015).

Flat parameter order (71,426 values): W1 (256 x 19, row = output unit),
b1 (256), W2 (256 x 256), b2 (256), W3 (2 x 256), b3 (2).

Inputs: the 19 features are mapped by t (asinh on the 16 Lanczos-coefficient
features, identity on the three log2 sizes) and standardised with fixed
per-feature means and scales.

Forward, with Wb = bf16(W) and xhat the standardised features:
    z1 = xhat Wb1^T + b1,  h1 = relu(z1)
    z2 = h1 Wb2^T + b2,    h2 = relu(z2)
    u  = h2 Wb3^T + b3,    u = (u0, u1) = (mean, log variance)
Loss (per batch of B): L = (1/B) sum 0.5 * (u1 + (r - u0)^2 exp(-u1)).
Gradients treat the BF16 rounding as the identity (straight-through) and are
taken with respect to the master weights.
"""
from __future__ import annotations

from typing import Dict, Tuple

import numpy as np

N_IN, N_HID, N_OUT = 19, 256, 2
SHAPES = [("W1", (N_HID, N_IN)), ("b1", (N_HID,)), ("W2", (N_HID, N_HID)), ("b2", (N_HID,)),
          ("W3", (N_OUT, N_HID)), ("b3", (N_OUT,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(theta: np.ndarray) -> Dict[str, np.ndarray]:
    out, o = {}, 0
    for name, shape in SHAPES:
        n = int(np.prod(shape))
        out[name] = np.asarray(theta[o:o + n], dtype=np.float64).reshape(shape)
        o += n
    return out


def pack(p: Dict[str, np.ndarray]) -> np.ndarray:
    return np.concatenate([np.asarray(p[name], dtype=np.float64).reshape(-1) for name, _ in SHAPES])


def bf16_round(x: np.ndarray) -> np.ndarray:
    """Round FP32 values to BF16 (round to nearest, ties to even); returns
    float64 holding the BF16 values exactly."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    u = (u + np.uint64(0x7FFF) + lsb) & np.uint64(0xFFFF0000)
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


N_COEF = 16


def input_transform(x: np.ndarray) -> np.ndarray:
    """asinh on the 16 Lanczos-coefficient features, identity on the three
    log2 subsystem sizes."""
    x = np.array(x, dtype=np.float64)
    x[..., :N_COEF] = np.arcsinh(x[..., :N_COEF])
    return x


def standardise(x: np.ndarray, mu: np.ndarray, sd: np.ndarray) -> np.ndarray:
    """xhat = (t(x) - mean) / scale with t = input_transform."""
    return (input_transform(x) - mu) / sd


def forward(theta: np.ndarray, xhat: np.ndarray, quantise: bool = True):
    p = unpack(theta)
    q = bf16_round if quantise else (lambda w: np.asarray(w, dtype=np.float64))
    w1, w2, w3 = q(p["W1"]), q(p["W2"]), q(p["W3"])
    x = np.asarray(xhat, dtype=np.float64)
    z1 = x @ w1.T + p["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ w2.T + p["b2"]
    h2 = np.maximum(z2, 0.0)
    u = h2 @ w3.T + p["b3"]
    cache = {"x": x, "z1": z1, "h1": h1, "z2": z2, "h2": h2, "w1": w1, "w2": w2, "w3": w3}
    return u, cache


def nll(u: np.ndarray, r: np.ndarray) -> float:
    d = np.asarray(r, dtype=np.float64) - u[:, 0]
    return float(np.mean(0.5 * (u[:, 1] + d * d * np.exp(-u[:, 1]))))


def loss_and_grad(theta: np.ndarray, xhat: np.ndarray, r: np.ndarray,
                  quantise: bool = True) -> Tuple[float, np.ndarray, np.ndarray]:
    """Returns (loss, flat gradient, network output u)."""
    u, c = forward(theta, xhat, quantise)
    B = u.shape[0]
    d = np.asarray(r, dtype=np.float64) - u[:, 0]
    ex = np.exp(-u[:, 1])
    du = np.empty_like(u)
    du[:, 0] = -d * ex / B
    du[:, 1] = 0.5 * (1.0 - d * d * ex) / B
    g = {}
    g["W3"] = du.T @ c["h2"]
    g["b3"] = du.sum(axis=0)
    dh2 = du @ c["w3"]
    dz2 = dh2 * (c["z2"] > 0.0)
    g["W2"] = dz2.T @ c["h1"]
    g["b2"] = dz2.sum(axis=0)
    dh1 = dz2 @ c["w2"]
    dz1 = dh1 * (c["z1"] > 0.0)
    g["W1"] = dz1.T @ c["x"]
    g["b1"] = dz1.sum(axis=0)
    return nll(u, r), pack(g), u


def adam_step(theta: np.ndarray, m: np.ndarray, v: np.ndarray, g: np.ndarray, t: int, lr: float,
              beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
    """One Adam update (step number t >= 1) with bias correction."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    theta = theta - lr * mhat / (np.sqrt(vhat) + eps)
    return theta, m, v

