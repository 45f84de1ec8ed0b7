"""Learned early stopping for TNSLQ (the project's addition; the paper has no
learned component).

A 19 -> 256 -> 256 -> 2 perceptron (the library's MLP kernels) reads, after
the first n_early Lanczos steps (4 to 8, fixed when the network is trained),
the probe means of d_A d_B alpha_1..n_early and d_A d_B beta_2..n_early+1
(each kind in eight slots, the unused ones zero) plus log2 d_A, log2 d_B,
log2 d_E, and predicts the residual between the converged estimate and the
n_early-step SLQ estimate E_early:
    mu = E_early + y_scale * u0,     sigma = y_scale * exp(u1 / 2).
At run time (tnslq_logneg_surrogate) the estimate stops after n_early steps
when sigma <= tol * max(|mu|, 1); otherwise the same Lanczos state continues
to the full step count.

Everything here is orchestration: instance drawing, the per-instance calls of
tnslq_logneg (whose alpha, beta and quadrature values are the training data),
the minibatch loop over tnslq_mlp_train, and checkpoint files.  Training and
inference arithmetic runs in the HIP kernels.

    python -m paper_1809_01685_amd.surrogate generate --n 20000 --out DIR
    python -m paper_1809_01685_amd.surrogate train --data DIR --early 5 --out DIR
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time
from dataclasses import dataclass, field
from typing import Dict, List, Optional

import numpy as np

from . import (MLP_NIN, MLP_NPARAMS, tnslq_logneg, tnslq_logneg_surrogate, tnslq_mlp_forward, tnslq_mlp_train,
               tnslq_mlp_loss_grad)

FEATURE_STEPS = 8          # n_early of a checkpoint that does not record it
SLOTS = 8                  # coefficient slots per kind in the network input
RECORD_STEPS = 9           # early estimates E_1..E_9 kept per training instance
WEIGHTS_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "surrogate_weights")


# ------------------------------------------------------------------ features
def coefficient_means(alpha: np.ndarray, beta: np.ndarray, d_a: int, d_b: int):
    """d_A d_B times the probe means of alpha_1..8 and of beta_2..9 from a
    run's (K, m) alpha and (K, m+1) beta (m >= 8)."""
    n = float(d_a * d_b)
    return n * alpha[:, :SLOTS].mean(axis=0), n * beta[:, 1:SLOTS + 1].mean(axis=0)


def features(am: np.ndarray, bm: np.ndarray, d_a, d_b, d_e, n_early: int) -> np.ndarray:
    """The 19 network inputs for rows of coefficient means (..., 8) read after
    n_early steps (same slots as the library's on-device feature kernel):
    the first n_early of each kind, the rest zero, then the log2 sizes."""
    am = np.asarray(am, dtype=np.float64)
    bm = np.asarray(bm, dtype=np.float64)
    out = np.zeros(am.shape[:-1] + (MLP_NIN,))
    out[..., :n_early] = am[..., :n_early]
    out[..., SLOTS:SLOTS + n_early] = bm[..., :n_early]
    out[..., 2 * SLOTS] = np.log2(d_a)
    out[..., 2 * SLOTS + 1] = np.log2(d_b)
    out[..., 2 * SLOTS + 2] = np.log2(d_e)
    return out


def features_from_coefficients(alpha: np.ndarray, beta: np.ndarray, d_a: int, d_b: int, d_e: int,
                               n_early: int = FEATURE_STEPS) -> np.ndarray:
    """The 19 network inputs from a run's (K, m) alpha and (K, m+1) beta."""
    am, bm = coefficient_means(alpha, beta, d_a, d_b)
    return features(am, bm, d_a, d_b, d_e, n_early)


def dataset_features(data: Dict[str, np.ndarray], n_early: int):
    """(X, E_early) of a generated dataset for a network reading n_early steps."""
    meta = data["meta"]
    d_a, d_b = 2.0 ** meta[:, 1], 2.0 ** meta[:, 2]
    d_e = 2.0 ** (meta[:, 0] - meta[:, 1] - meta[:, 2])
    X = features(data["A"], data["B"], d_a, d_b, d_e, n_early)
    return X, data["E"][:, n_early - 1]


def input_transform(X: np.ndarray) -> np.ndarray:
    """The fixed map applied before standardisation (the kernel applies the
    same): asinh on the 16 Lanczos-coefficient features, which span many
    decades (nearly pure rho_AB has d_A d_B alpha ~ d_A d_B), identity on the
    three log2 sizes.  Used here only to compute the standardisation
    constants."""
    X = np.array(X, dtype=np.float64)
    X[..., :16] = np.arcsinh(X[..., :16])
    return X


def estimate_at(beta: np.ndarray, F: np.ndarray, j: int) -> float:
    """SLQ estimate log2 mean(beta_1^2 F_j) after j steps."""
    return float(np.log2(np.mean(beta[:, 0] ** 2 * F[:, j - 1])))


# ------------------------------------------------------------------ instances
@dataclass
class Instance:
    n_qubits: int
    a: List[int]
    b: List[int]
    kind: str
    depth: int
    seed: int

    @property
    def dims(self):
        ne = self.n_qubits - len(self.a) - len(self.b)
        return 1 << len(self.a), 1 << len(self.b), 1 << ne


def draw_instance(rng: np.random.Generator, l_min: int = 16, l_max: int = 22) -> Instance:
    import tnslq_inputs as ti
    L = int(rng.integers(l_min, l_max + 1))
    a, b = ti.random_contiguous_partition(L, rng)
    kind = "haar" if rng.random() < 0.5 else "brickwork"
    depth = int(rng.integers(1, 13)) if kind == "brickwork" else 0
    return Instance(L, a, b, kind, depth, int(rng.integers(0, 2**31)))


def instance_state(inst: Instance, device):
    import torch
    import tnslq_inputs as ti
    if inst.kind == "haar":
        return ti.haar_state_torch(inst.n_qubits, inst.seed, device, torch.complex64)
    return ti.brickwork_state_torch(inst.n_qubits, inst.depth, inst.seed, device, torch.complex64)


def run_instance(inst: Instance, device, n_probes=32, n_steps=40, precision="bf16x3", seed=0) -> Dict[str, object]:
    psi = instance_state(inst, device)
    r = tnslq_logneg(psi, inst.n_qubits, inst.a, inst.b, n_probes, n_steps, precision=precision, seed=seed)
    d_a, d_b, d_e = inst.dims
    am, bm = coefficient_means(r["alpha"], r["beta"], d_a, d_b)
    return {"A": am, "B": bm, "E": np.array([estimate_at(r["beta"], r["F"], j) for j in range(1, RECORD_STEPS + 1)]),
            "e_full": float(r["logneg"]), "se_full": float(r["logneg_se"]), "steps_min": int(r["steps_min"]),
            "dims": (d_a, d_b, d_e)}


def generate(n: int, seed: int, device, n_probes=32, n_steps=40, precision="bf16x3", l_min=16, l_max=22,
             log_every=500) -> Dict[str, np.ndarray]:
    """n method-generated training instances: coefficient means of the first
    eight steps, early estimates E_1..E_9 and the full-SLQ label, so that a
    network for any n_early in 4..8 can be trained from one set."""
    rng = np.random.default_rng(seed)
    A = np.zeros((n, SLOTS))
    B = np.zeros((n, SLOTS))
    E = np.zeros((n, RECORD_STEPS))
    ef = np.zeros(n)
    meta = []
    t0 = time.time()
    for i in range(n):
        inst = draw_instance(rng, l_min, l_max)
        out = run_instance(inst, device, n_probes, n_steps, precision, seed=inst.seed)
        A[i], B[i], E[i], ef[i] = out["A"], out["B"], out["E"], out["e_full"]
        meta.append([inst.n_qubits, len(inst.a), len(inst.b), inst.depth, int(inst.kind == "haar"), inst.seed])
        if log_every and (i + 1) % log_every == 0:
            print(f"[surrogate] generated {i + 1}/{n} instances in {time.time() - t0:.1f} s", flush=True)
    return {"A": A, "B": B, "E": E, "e_full": ef, "meta": np.array(meta, dtype=np.int64),
            "seconds": np.array(time.time() - t0)}


# ------------------------------------------------------------------ model
@dataclass
class Model:
    params: np.ndarray                 # float32[71426]
    norm: np.ndarray                   # float32[38]: feature means then scales
    y_scale: float
    meta: Dict[str, object] = field(default_factory=dict)

    @property
    def feature_steps(self) -> int:
        return int(self.meta.get("feature_steps", FEATURE_STEPS))

    def save(self, path: str) -> None:
        os.makedirs(path, exist_ok=True)
        self.params.astype("<f4").tofile(os.path.join(path, "params.bin"))
        self.norm.astype("<f4").tofile(os.path.join(path, "norm.bin"))
        with open(os.path.join(path, "model.json"), "w") as f:
            json.dump({"n_params": int(self.params.size), "y_scale": float(self.y_scale), **self.meta}, f, indent=1)

    @staticmethod
    def load(path: str = WEIGHTS_DIR) -> "Model":
        with open(os.path.join(path, "model.json")) as f:
            meta = json.load(f)
        params = np.fromfile(os.path.join(path, "params.bin"), dtype="<f4")
        norm = np.fromfile(os.path.join(path, "norm.bin"), dtype="<f4")
        if params.size != MLP_NPARAMS or norm.size != 2 * MLP_NIN:
            raise ValueError(f"bad checkpoint in {path}")
        y_scale = float(meta.pop("y_scale"))
        return Model(params, norm, y_scale, meta)

    def device_tensors(self, device):
        import torch
        return (torch.from_numpy(np.ascontiguousarray(self.params)).to(device),
                torch.from_numpy(np.ascontiguousarray(self.norm)).to(device))


def train(data: Dict[str, np.ndarray], device, n_early=FEATURE_STEPS, seed=0, epochs=150, batch=256, lr=1e-3,
          val_frac=0.1, log=True) -> Model:
    """Fit the network to (E_full - E_early) / y_scale with the library's
    kernels; the validation split is by instance (the last val_frac of a
    seeded permutation)."""
    import torch
    import tnslq_inputs as ti
    t_start = time.time()
    X, e8 = dataset_features(data, n_early)
    ef = data["e_full"]
    n = X.shape[0]
    rng = np.random.default_rng(seed)
    perm = rng.permutation(n)
    n_val = max(1, int(round(val_frac * n)))
    tr, va = perm[:-n_val], perm[-n_val:]
    resid = ef - e8
    y_scale = float(np.std(resid[tr])) or 1.0
    Xt = input_transform(X)
    mu = Xt[tr].mean(axis=0)
    sd = Xt[tr].std(axis=0)
    sd[sd < 1e-6] = 1.0
    norm = np.concatenate([mu, sd]).astype(np.float32)
    r = (resid / y_scale).astype(np.float32)

    th = torch.from_numpy(ti.mlp_init_params(seed)).to(device)
    m = torch.zeros_like(th)
    v = torch.zeros_like(th)
    xd = torch.from_numpy(X.astype(np.float32)).to(device)
    rd = torch.from_numpy(r).to(device)
    nd = torch.from_numpy(norm).to(device)
    t = 1
    best = (float("inf"), None)
    n_tr = tr.size - tr.size % batch
    for ep in range(epochs):
        idx = torch.from_numpy(rng.permutation(tr)[:n_tr].astype(np.int32)).to(device)
        t = tnslq_mlp_train(th, m, v, nd, xd, rd, idx, batch, t, lr)
        if (ep + 1) % 10 == 0 or ep == epochs - 1:
            vi = torch.from_numpy(va).to(device)
            vl = float(tnslq_mlp_loss_grad(th, nd, xd[vi], rd[vi])[0].cpu())
            if vl < best[0]:
                best = (vl, th.clone())
            if log:
                print(f"[surrogate] epoch {ep + 1}: validation NLL {vl:.4f}", flush=True)
    params = best[1].cpu().numpy()
    torch.cuda.synchronize(device)
    return Model(params, norm, y_scale, {"feature_steps": int(n_early), "n_train": int(tr.size), "n_val": int(n_val),
                                         "epochs": epochs, "batch": batch, "lr": lr, "seed": seed, "val_nll": best[0],
                                         "train_seconds": time.time() - t_start,
                                         "val_index": [int(i) for i in va]})


def predict(model: Model, X: np.ndarray, e8: np.ndarray, device):
    """(mu, sigma) for feature rows X with early estimates e8 (after the
    model's feature_steps steps)."""
    import torch
    p, nd = model.device_tensors(device)
    u = tnslq_mlp_forward(p, nd, torch.from_numpy(np.ascontiguousarray(X, dtype=np.float32)).to(device)).cpu().numpy()
    mu = e8 + model.y_scale * u[:, 0].astype(np.float64)
    sigma = model.y_scale * np.exp(0.5 * u[:, 1].astype(np.float64))
    return mu, sigma


def surrogate_logneg(model: Model, psi, n_qubits, a, b, n_probes, n_steps, tol=0.01, precision="bf16x3", seed=0,
                     **kw):
    p, nd = model.device_tensors(psi.device)
    return tnslq_logneg_surrogate(psi, n_qubits, a, b, n_probes, n_steps, p, nd, model.y_scale, tol=tol,
                                  early_steps=model.feature_steps, precision=precision, seed=seed, **kw)


# ------------------------------------------------------------------ CLI
def _main(argv=None):
    import torch
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    g = sub.add_parser("generate")
    g.add_argument("--n", type=int, default=20000)
    g.add_argument("--seed", type=int, default=1)
    g.add_argument("--out", required=True)
    g.add_argument("--precision", default="bf16x3")
    g.add_argument("--l-min", type=int, default=16)
    g.add_argument("--l-max", type=int, default=22)
    t = sub.add_parser("train")
    t.add_argument("--data", required=True)
    t.add_argument("--out", default=WEIGHTS_DIR)
    t.add_argument("--epochs", type=int, default=150)
    t.add_argument("--seed", type=int, default=0)
    t.add_argument("--early", type=int, default=FEATURE_STEPS, help="Lanczos steps the network reads (4-8)")
    args = ap.parse_args(argv)
    dev = torch.device("cuda:0")
    if args.cmd == "generate":
        os.makedirs(args.out, exist_ok=True)
        d = generate(args.n, args.seed, dev, precision=args.precision, l_min=args.l_min, l_max=args.l_max)
        np.savez(os.path.join(args.out, "dataset.npz"), **d)
        print(f"[surrogate] wrote {args.n} instances to {args.out} in {float(d['seconds']):.1f} s", flush=True)
    else:
        path = args.data if args.data.endswith(".npz") else os.path.join(args.data, "dataset.npz")
        with np.load(path) as f:
            d = {k: f[k] for k in f.files}
        model = train(d, dev, n_early=args.early, seed=args.seed, epochs=args.epochs)
        model.save(args.out)
        va = np.array(model.meta["val_index"])
        X, e_early = dataset_features(d, model.feature_steps)
        mu, sigma = predict(model, X[va], e_early[va], dev)
        err_mlp = np.abs(mu - d["e_full"][va])
        err_e8 = np.abs(e_early[va] - d["e_full"][va])
        print(json.dumps({"n_early": model.feature_steps, "train_seconds": model.meta["train_seconds"],
                          "val_mae_mlp": float(err_mlp.mean()), "val_mae_early": float(err_e8.mean()),
                          "val_median_mlp": float(np.median(err_mlp)), "val_median_early": float(np.median(err_e8)),
                          "accept_rate": float(np.mean(sigma <= 0.01 * np.maximum(np.abs(mu), 1.0)))}))


if __name__ == "__main__":
    _main(sys.argv[1:])
