"""Parity and properties at the full workload sizes.

* 20-qubit Haar state, A = 0-5, B = 8-13 (d_A d_B = 4096), 32 probes, 40
  steps with reorthogonalisation: against the explicit-operator oracle on the
  same probes (FP32 on complex64 and FP64 on complex128), and the SLQ
  estimate against the exact eigensolve.
* 30-qubit Haar state, E = 0-3, A = 4-16, B = 17-29 (a 26-qubit rho_AB, the
  benchmarked workload), split-BF16: no explicit oracle exists (2^52 operator
  entries), so sampled matvec outputs are computed by the oracle one at a time,
  Hermiticity is checked on a vector pair, and the estimate is compared with
  Eq. 6 of Sec. VII.A.
"""
import numpy as np
import pytest

import tnslq_inputs as ti
from oracle import analytic, exact, probes, slq

pytestmark = pytest.mark.gpu
T = pytest.importorskip("paper_1809_01685_amd")

L20, A20, B20 = 20, list(range(6)), list(range(8, 14))


@pytest.fixture(scope="module")
def haar20():
    return ti.haar_state(L20, 0)


@pytest.mark.parametrize("operator", ["lazy", "explicit"])
@pytest.mark.parametrize("prec,dtype", [("fp32", np.complex64), ("fp64", np.complex128)])
def test_haar20_matches_oracle_on_same_probes(dev, haar20, prec, dtype, operator):
    import torch
    psi = haar20.astype(dtype)
    psi_t = torch.from_numpy(psi).to(dev)
    g = T.tnslq_logneg(psi_t, L20, A20, B20, 32, 40, reorth=True, precision=prec, seed=7, operator=operator)
    assert g["explicit_operator"] == (operator == "explicit")
    P = exact.regroup(psi.astype(np.complex128), L20, A20, B20)
    R = exact.rho_pt(P)
    X = probes.rademacher_probes(7, 32, 4096)
    o = slq.slq(lambda v: R @ v, X, 40, reorth=True)
    o.update(slq.hutchinson_stats(o["G"]))
    tol = (1e-4 if prec == "fp32" else 1e-10) * max(abs(o["logneg"]), 1.0)
    print(prec, g["logneg"], o["logneg"], g["logneg"] - o["logneg"])
    assert abs(g["logneg"] - o["logneg"]) <= tol
    scale = np.max(np.abs(o["alpha"]))
    k = 40 if prec == "fp64" else 8
    atol = 1e-9 if prec == "fp64" else 1e-5
    assert np.max(np.abs(g["alpha"][:, :k] - o["alpha"][:, :k])) <= atol * scale
    # and the estimate agrees with the exact trace norm within its error bar
    e = exact.logneg_exact(P)
    assert abs(g["logneg"] - e) <= 4 * g["logneg_se"] + 2e-3 * e


def test_haar20_matvec_fp32_block(dev, haar20):
    import torch
    psi = haar20.astype(np.complex64)
    P = exact.regroup(psi.astype(np.complex128), L20, A20, B20)
    X = ti.random_vectors(32, 4096, seed=3)
    Y = T.tnslq_ptmatvec(torch.from_numpy(psi).to(dev), L20, A20, B20, torch.from_numpy(X).to(dev),
                         precision="fp32").cpu().numpy()
    ref = exact.pt_matvec_explicit(P, X)
    assert np.linalg.norm(Y - ref) / np.linalg.norm(ref) <= 1e-6


L30, A30, B30 = 30, list(range(4, 17)), list(range(17, 30))


@pytest.fixture(scope="module")
def haar30(dev):
    import torch
    return ti.haar_state_torch(L30, 0, dev, torch.complex64)


def test_haar30_sampled_matvec_outputs(dev, haar30):
    import torch
    X = ti.random_vectors(2, 1 << 26, seed=11)
    Y = T.tnslq_ptmatvec(haar30, L30, A30, B30, torch.from_numpy(X).to(dev), precision="bf16x3")
    # Hermiticity on the pair: <x0, Y x1> = conj <x1, Y x0>
    Yh = Y.cpu().numpy()
    lhs = np.vdot(X[0], Yh[1])
    rhs = np.conj(np.vdot(X[1], Yh[0]))
    assert abs(lhs - rhs) <= 1e-4 * np.linalg.norm(X[0]) * np.linalg.norm(Yh[1])
    # outputs y[a, b] of vector 0 for a few rows in two columns, one at a time
    psi = haar30.cpu().numpy()
    slab = lambda c: psi[c << 26:(c + 1) << 26].reshape(1 << 13, 1 << 13)  # noqa: E731
    x0 = X[0].reshape(1 << 13, 1 << 13)
    y0 = Yh[0].reshape(1 << 13, 1 << 13)
    rms = np.sqrt(np.mean(np.abs(Yh[0]) ** 2))
    rng = np.random.default_rng(5)
    entries = [(int(rng.integers(0, 1 << 13)), col) for col in (17, 6001) for _ in range(4)]
    want = exact.pt_matvec_entries_from_slabs(slab, 16, x0, entries)
    got = np.array([y0[a, b] for a, b in entries])
    # per entry: 5x the norm-wise BF16X3 bound, relative to the RMS output
    assert np.max(np.abs(got - want)) <= 1.5e-4 * rms, (got, want)


def test_haar30_estimate_near_random_state_value(dev, haar30):
    g = T.tnslq_logneg(haar30, L30, A30, B30, 2, 12, precision="bf16x3", seed=3)
    want = analytic.random_state_logneg(1 << 13, 1 << 13, 16)
    assert abs(g["logneg"] - want) <= 0.01 * want
