"""The learned early stop's decision after the first Lanczos steps (the
project's addition to Algorithm 1 of Sec. III; the paper has no learned
part).

Oracle, test infrastructure only.

After n_early Lanczos steps (4 to 8, the value the network was trained
with) of a block of N probes:

  * features (19 values): eight slots of probe means of d_A d_B alpha_j
    (j = 1..n_early, the rest zero), eight of d_A d_B beta_j (j =
    2..n_early+1, the rest zero; beta_1 = ||phi|| is the same for every probe
    and is left out), then log2 d_A, log2 d_B, log2 d_E in the caller's roles;
  * the network's input: the features in single precision (the network takes
    FP32 inputs), mapped by asinh (the 16 coefficient features) and
    standardised with the fixed means and scales of `norm`;
  * the network (oracle.mlp.forward, BF16-rounded weights) gives (u0, u1);
  * the early estimate E_early = log2 mean_n ||phi_n||^2 F_{n_early},n (the
    plain quadrature of T_{n_early});
  * mu = E_early + y_scale u0 and sigma = y_scale exp(u1 / 2);
  * the early result is accepted when both are finite and
    sigma <= tol max(|mu|, 1); otherwise the run goes on to full SLQ.
"""
from __future__ import annotations

from typing import Dict

import numpy as np

from . import mlp, step_difference

N_EARLY = 8
SLOTS = 8   # coefficient slots per kind in the network input


def block_features(alpha: np.ndarray, beta: np.ndarray, d_a: int, d_b: int, d_e: int,
                   n_early: int = N_EARLY) -> np.ndarray:
    """The 19 inputs from a block's alpha (N x m) and beta (N x (m+1), beta_1
    first): N' alpha_1..n_early and N' beta_2..n_early+1 averaged over the
    probes (N' = d_A d_B), each kind zero padded to eight slots, then log2
    d_A, log2 d_B, log2 d_E."""
    alpha = np.asarray(alpha, dtype=np.float64)
    beta = np.asarray(beta, dtype=np.float64)
    if not 1 <= n_early <= SLOTS:
        raise ValueError("n_early outside the network's eight slots")
    if alpha.shape[1] < n_early or beta.shape[1] < n_early + 1:
        raise ValueError("fewer Lanczos coefficients than the network reads")
    n = float(d_a) * float(d_b)
    fa = np.zeros(SLOTS)
    fb = np.zeros(SLOTS)
    fa[:n_early] = n * np.mean(alpha[:, :n_early], axis=0)
    fb[:n_early] = n * np.mean(beta[:, 1:n_early + 1], axis=0)
    return np.concatenate([fa, fb, [np.log2(d_a), np.log2(d_b), np.log2(d_e)]])


def network_input(features: np.ndarray, norm: np.ndarray) -> np.ndarray:
    """Standardised network input from the features and the 38 constants of
    `norm` (19 means, then 19 scales)."""
    x = np.asarray(features, dtype=np.float32).astype(np.float64)
    norm = np.asarray(norm, dtype=np.float64)
    k = mlp.N_IN
    return mlp.standardise(x, norm[:k], norm[k:2 * k])


def decision(theta: np.ndarray, norm: np.ndarray, y_scale: float, alpha: np.ndarray, beta: np.ndarray,
             F: np.ndarray, d_a: int, d_b: int, d_e: int, tol: float, n_early: int = N_EARLY) -> Dict[str, object]:
    """The surrogate's outcome after n_early steps: features, network output
    (u0, u1), E_early, mu, sigma and whether the early result is accepted."""
    f = block_features(alpha, beta, d_a, d_b, d_e, n_early)
    xhat = network_input(f, norm)
    u, _ = mlp.forward(np.asarray(theta, dtype=np.float64), xhat[None, :])
    u0, u1 = float(u[0, 0]), float(u[0, 1])
    e_early = step_difference.block_estimate(beta, F, n_early)["logneg"]
    y = float(np.float32(y_scale))
    mu = e_early + y * u0
    sigma = y * float(np.exp(0.5 * u1))
    accept = bool(np.isfinite(mu) and np.isfinite(sigma) and sigma <= tol * max(abs(mu), 1.0))
    return {"features": f, "u": (u0, u1), "e_early": e_early, "mu": mu, "sigma": sigma, "accept": accept}
