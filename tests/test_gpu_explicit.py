"""GPU parity of the explicit operator (Sec. V, intermediary (iii)) against the
oracle, through the C ABI.

* tnslq_rho_pt forms rho_AB^{T_B} in FP64 (a product over d_E terms, then the
  exchange of B's indices); every entry matches the oracle's partial transpose
  of P P^dagger to 1e-13 of the largest entry.
* tnslq_logneg with operator="explicit" runs Algorithm 1 on that matrix; in
  FP64 its Lanczos coefficients and estimates match the oracle's on the same
  probes to 1e-10 relative, in the reduced precisions the estimate to
  1e-4 max(|E|, 1).
* operator="auto" takes the explicit form where its padded multiply-adds are
  fewer (the 20-qubit workload) and the lazy one elsewhere.
"""
import numpy as np
import pytest

import tnslq_inputs as ti
from oracle import exact, slq

pytestmark = pytest.mark.gpu

T = pytest.importorskip("paper_1809_01685_amd")

LOGNEG_TOL = {"fp64": 1e-10, "fp32": 1e-4, "bf16x6": 1e-4, "bf16x3": 1e-4}

PARTS = [
    (6, [0, 1, 2], [3, 4, 5]),          # empty environment (pure state), d_A d_B = 64
    (8, [1, 5], [0, 3, 6]),             # |B| > |A|, non-contiguous: no role exchange here
    (9, [0, 2, 4], [6, 8]),
    (10, [0, 1, 2], [3, 4, 5]),         # the 10-qubit workload's partition
    (12, [7], [2]),                     # d_A d_B = 4: one brick row, mostly padding
    (11, [0, 1, 2, 3, 4], [6, 7, 8, 9, 10]),
    (14, [13, 0, 6, 2, 9, 4], [1, 12, 3, 11, 5, 7]),   # d_A d_B = 4096, unordered qubits
]


def _dev_state(psi_np, dtype, dev):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(psi_np.astype(dtype))).to(dev)
    return t, t.cpu().numpy().astype(np.complex128)


@pytest.mark.parametrize("dtype", [np.complex128, np.complex64])
@pytest.mark.parametrize("L,a,b", PARTS)
def test_rho_pt_matches_oracle(dev, L, a, b, dtype):
    psi_t, psi_o = _dev_state(ti.haar_state(L, L + 2), dtype, dev)
    R = T.tnslq_rho_pt(psi_t, L, a, b).cpu().numpy()
    want = exact.rho_pt(exact.regroup(psi_o, L, a, b))
    scale = np.max(np.abs(want))
    assert R.shape == want.shape
    assert np.max(np.abs(R - want)) <= 1e-13 * scale
    # Hermitian, trace = ||psi||^2 (the partial transpose keeps the trace; the
    # complex64 amplitudes are normalised only to their rounding)
    assert np.max(np.abs(R - R.conj().T)) <= 1e-13 * scale
    assert np.trace(R).real == pytest.approx(float(np.vdot(psi_o, psi_o).real), abs=1e-12)


@pytest.mark.parametrize("L,a,b", PARTS)
def test_explicit_logneg_matches_oracle_fp64(dev, L, a, b):
    psi_t, psi_o = _dev_state(ti.haar_state(L, L), np.complex128, dev)
    K, m = 6, 12
    g = T.tnslq_logneg(psi_t, L, a, b, K, m, precision="fp64", seed=3, operator="explicit")
    o = slq.slq_logneg(psi_o, L, a, b, K, m, seed=3)
    assert g["explicit_operator"] == 1 and g["swapped_ab"] == 0 and g["streamed"] == 0
    assert np.array_equal(g["steps"], o["steps"])
    scale = np.max(np.abs(o["alpha"]))
    # coefficients up to each probe's stop (past a breakdown both sides hold 0)
    assert np.max(np.abs(g["alpha"] - o["alpha"])) <= 1e-10 * scale
    assert np.array_equal(g["beta"][:, 0], o["beta"][:, 0])
    assert np.max(np.abs(g["beta"][:, 1:] - o["beta"][:, 1:])) <= 1e-10 * np.max(np.abs(o["beta"][:, 1:]))
    assert np.allclose(g["G"], o["G"], rtol=1e-10, atol=1e-14)
    assert g["logneg"] == pytest.approx(o["logneg"], abs=1e-10 * max(abs(o["logneg"]), 1.0))


@pytest.mark.parametrize("prec,dtype", [("fp32", np.complex64), ("fp32", np.complex128), ("bf16x3", np.complex64),
                                        ("bf16x6", np.complex64)])
@pytest.mark.parametrize("L,a,b", [PARTS[1], PARTS[3], PARTS[6]])
def test_explicit_logneg_reduced_precisions(dev, L, a, b, prec, dtype):
    # with reorthogonalisation: without it, 16 steps on a 32-dimensional space
    # lose orthogonality, and a 1e-5 perturbation of the matvec then moves the
    # quadrature by ~1e-3 on either side of the FP64 trajectory (reproduced by
    # emulating the split-BF16 rounding on the CPU)
    psi_t, psi_o = _dev_state(ti.haar_state(L, L + 5), dtype, dev)
    K, m = 8, 16
    g = T.tnslq_logneg(psi_t, L, a, b, K, m, reorth=True, precision=prec, seed=2, operator="explicit")
    o = slq.slq_logneg(psi_o, L, a, b, K, m, seed=2, reorth=True)
    tol = LOGNEG_TOL[prec] * max(abs(o["logneg"]), 1.0)
    print(L, prec, np.dtype(dtype).name, g["logneg"], o["logneg"], g["logneg"] - o["logneg"])
    assert abs(g["logneg"] - o["logneg"]) <= tol


def test_explicit_and_lazy_agree_on_same_probes(dev):
    import torch
    L, a, b = 13, [0, 1, 2, 3, 4], [7, 8, 9, 10]
    psi_t = torch.from_numpy(ti.haar_state(L, 4)).to(dev)
    e = T.tnslq_logneg(psi_t, L, a, b, 16, 20, reorth=True, precision="fp64", seed=9, operator="explicit")
    z = T.tnslq_logneg(psi_t, L, a, b, 16, 20, reorth=True, precision="fp64", seed=9, operator="lazy")
    scale = np.max(np.abs(z["alpha"]))
    assert np.max(np.abs(e["alpha"] - z["alpha"])) <= 1e-11 * scale
    assert np.max(np.abs(e["beta"] - z["beta"])) <= 1e-11 * scale
    assert e["logneg"] == pytest.approx(z["logneg"], abs=1e-11)
    # timing fields: one dense product per step; the first contraction's
    # interval is two back-to-back events (a few microseconds per step)
    assert e["n_contract_launches"] == e["steps_done"] and e["t_contract1_ms"] <= 0.01 * e["steps_done"]


def test_auto_takes_the_cheaper_form(dev):
    import torch
    # 20 qubits, A = 0-5, B = 8-13 (d_A d_B = 4096, d_E = 256), K = 32, 40 steps
    psi_t = torch.from_numpy(ti.haar_state(20, 1).astype(np.complex64)).to(dev)
    r = T.tnslq_logneg(psi_t, 20, list(range(6)), list(range(8, 14)), 32, 40, precision="fp32", seed=0,
                       want_arrays=False)
    assert r["explicit_operator"] == 1
    # d_A d_B = 2^16 exceeds the explicit form's limit
    r = T.tnslq_logneg(psi_t, 20, list(range(8)), list(range(8, 16)), 4, 6, precision="fp32", seed=0,
                       want_arrays=False)
    assert r["explicit_operator"] == 0
    # K d_B <= 8: the streaming passes
    r = T.tnslq_logneg(psi_t, 20, list(range(6)), [10], 2, 6, precision="fp32", seed=0, want_arrays=False)
    assert r["explicit_operator"] == 0 and r["streamed"] == 1
    del psi_t
    torch.cuda.empty_cache()
