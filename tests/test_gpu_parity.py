"""GPU parity of the HIP path against the FP64 oracle, through the C ABI.

Tolerances (norm-wise relative error over the whole block unless stated):
  * matvec FP64: 1e-12 (FP64 rounding of a few thousand-term sums).
  * matvec FP32 and BF16X6: 1e-6 (FP32 operands carry 2^-24 relative error,
    sums run in blocks of at most one tile and are merged in FP64).
  * matvec BF16X3: 3e-5 (a hi + lo split keeps 16 significant bits, 2^-17
    per operand; four rounded operands along the two contractions, plus FP32
    sums, bound the relative error by about 4 * 2^-17 = 3e-5).
  * logneg on the same probes: |dE| <= 1e-4 * max(|E|, 1) for the reduced
    precisions, 1e-10 * max(|E|, 1) for FP64.
"""
import numpy as np
import pytest

import tnslq_inputs as ti
from oracle import exact, probes, slq

pytestmark = pytest.mark.gpu

T = pytest.importorskip("paper_1809_01685_amd")

MATVEC_TOL = {"fp64": 1e-12, "fp32": 1e-6, "bf16x6": 1e-6, "bf16x3": 3e-5}
LOGNEG_TOL = {"fp64": 1e-10, "fp32": 1e-4, "bf16x6": 1e-4, "bf16x3": 1e-4}


def _dev_state(psi_np, dtype, dev):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(psi_np.astype(dtype))).to(dev)
    # the oracle sees the same rounded amplitudes
    return t, t.cpu().numpy().astype(np.complex128)


def _relerr(y, ref):
    return float(np.linalg.norm(y - ref) / np.linalg.norm(ref))


def test_probe_generator_bit_exact(dev):
    X = T.tnslq_probes(seed=7, probe_offset=3, n_probes=5, d=1000, device=dev).cpu().numpy()
    want = probes.rademacher_probes(7, 5, 1000, probe_offset=3)
    assert np.array_equal(X, want)


PARTS = [
    (6, [0, 1, 2], [3, 4, 5]),          # empty environment
    (8, [1, 5], [0, 3, 6]),             # |B| > |A|: roles swapped, non-contiguous
    (9, [0, 2, 4], [6, 8]),             # |B| < |A|
    (10, [0, 1, 2], [3, 4, 5]),         # the 10-qubit workload's partition
    (12, [7], [2]),                     # d_A = d_B = 2, d_E = 1024
    (11, [0, 1, 2, 3, 4], [6, 7, 8, 9, 10]),
    (14, list(range(6)), list(range(8, 14))),
    (13, list(range(9)), [10, 11]),     # d_B d_E = 16: the first contraction splits along a'
    (14, [0, 1, 2], [3, 4, 5]),         # d_B = 8, d_E = 256: the intermediary leaves the split
                                        # contraction through LDS with one row per environment index
]


@pytest.mark.parametrize("prec,dtype", [("fp64", np.complex128), ("fp32", np.complex64), ("fp32", np.complex128),
                                        ("bf16x3", np.complex64), ("bf16x6", np.complex64)])
@pytest.mark.parametrize("L,a,b", PARTS)
def test_ptmatvec_matches_explicit_operator(dev, L, a, b, prec, dtype):
    import torch
    psi_t, psi_np = _dev_state(ti.haar_state(L, L), dtype, dev)
    P = exact.regroup(psi_np, L, a, b)
    dab = P.shape[0] * P.shape[1]
    for K in (1, 3, 32):
        X = ti.random_vectors(K, dab, seed=K)
        Y = T.tnslq_ptmatvec(psi_t, L, a, b, torch.from_numpy(X).to(dev), precision=prec).cpu().numpy()
        ref = exact.pt_matvec_explicit(P, X)
        err = _relerr(Y, ref)
        print(f"L={L} a={a} b={b} {prec} {np.dtype(dtype).name} K={K}: matvec rel err {err:.2e}")
        assert err <= MATVEC_TOL[prec], (K, err)


def _logneg_case(dev, psi_np, L, a, b, K, m, prec, dtype, reorth, seed, operator="lazy"):
    psi_t, psi_o = _dev_state(psi_np, dtype, dev)
    g = T.tnslq_logneg(psi_t, L, a, b, K, m, reorth=reorth, precision=prec, seed=seed, operator=operator)
    assert g["explicit_operator"] == (operator == "explicit")
    o = slq.slq_logneg(psi_o, L, a, b, K, m, seed=seed, reorth=reorth)
    return g, o


@pytest.mark.parametrize("operator", ["lazy", "explicit"])
@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_logneg_matches_oracle_small_haar(dev, prec, operator):
    # 10-qubit Haar state, A = 0-2, B = 3-5; 16 probes, 20 steps.
    dtype = np.complex128 if prec == "fp64" else np.complex64
    g, o = _logneg_case(dev, ti.haar_state(10, 0), 10, [0, 1, 2], [3, 4, 5], 16, 20, prec, dtype, False, 0,
                        operator)
    tol = LOGNEG_TOL[prec] * max(abs(o["logneg"]), 1.0)
    print(prec, g["logneg"], o["logneg"], g["logneg"] - o["logneg"])
    assert abs(g["logneg"] - o["logneg"]) <= tol
    assert np.array_equal(g["steps"], o["steps"])
    # recurrence coefficients agree while the arithmetic difference is small
    scale = np.max(np.abs(o["alpha"]))
    k_cmp = 20 if prec == "fp64" else 6
    atol = 1e-10 if prec == "fp64" else 1e-4
    assert np.max(np.abs(g["alpha"][:, :k_cmp] - o["alpha"][:, :k_cmp])) <= atol * scale
    assert np.max(np.abs(g["beta"][:, :k_cmp + 1] - o["beta"][:, :k_cmp + 1])) <= atol * scale
    if prec == "fp64":
        assert np.allclose(g["G"], o["G"], rtol=1e-10, atol=0)
        assert np.allclose(g["F"], o["F"], rtol=1e-10, atol=0)
        assert g["logneg_se"] == pytest.approx(o["logneg_se"], rel=1e-8)


def test_logneg_swapped_roles_match_oracle(dev):
    # |B| > |A| exchanges the roles on the device; the conjugated probes keep
    # the Krylov coefficients identical to the oracle's.
    L, a, b = 9, [4, 1], [0, 6, 7]
    g, o = _logneg_case(dev, ti.haar_state(L, 3), L, a, b, 5, 12, "fp64", np.complex128, False, 11)
    assert g["swapped_ab"] == 1
    assert np.allclose(g["alpha"], o["alpha"], rtol=0, atol=1e-12 * np.max(np.abs(o["alpha"])))
    assert g["logneg"] == pytest.approx(o["logneg"], abs=1e-10)


@pytest.mark.parametrize("operator", ["lazy", "explicit"])
def test_logneg_reorth_matches_oracle(dev, operator):
    L, a, b = 12, [0, 1, 2, 3], [6, 7, 8]
    g, o = _logneg_case(dev, ti.haar_state(L, 5), L, a, b, 4, 24, "fp64", np.complex128, True, 2, operator)
    assert np.allclose(g["alpha"], o["alpha"], rtol=0, atol=1e-10 * np.max(np.abs(o["alpha"])))
    assert np.allclose(g["beta"], o["beta"], rtol=0, atol=1e-10 * np.max(np.abs(o["alpha"])))
    assert g["logneg"] == pytest.approx(o["logneg"], abs=1e-9)


@pytest.mark.parametrize("operator", ["lazy", "explicit"])
def test_bell_pair_and_product_state(dev, operator):
    L = 6
    g, _ = _logneg_case(dev, ti.bell_pair_state(L, 1, 4), L, [0, 1], [3, 4], 6, 10, "fp64", np.complex128, False, 2,
                        operator)
    assert g["logneg"] == pytest.approx(1.0, abs=1e-12)
    assert np.all(g["steps"] <= 3)
    assert np.allclose(g["G"], 2.0, atol=1e-12)
    g, _ = _logneg_case(dev, ti.basis_product_state(L, [0, 1, 1, 0, 1, 0]), L, [0, 2], [3, 5], 4, 6, "fp32",
                        np.complex64, False, 0, operator)
    assert g["logneg"] == pytest.approx(0.0, abs=1e-6)


@pytest.mark.parametrize("operator", ["lazy", "explicit"])
def test_pure_state_schmidt_formula(dev, operator):
    # empty environment: E = 2 log2 sum of singular values of psi as d_A x d_B
    L, a, b = 8, [0, 1, 2, 3], [4, 5, 6, 7]
    psi = ti.haar_state(L, 9)
    s = np.linalg.svd(psi.reshape(16, 16), compute_uv=False)
    want = 2 * np.log2(np.sum(s))
    g, o = _logneg_case(dev, psi, L, a, b, 64, 40, "fp64", np.complex128, True, 4, operator)
    assert g["logneg"] == pytest.approx(o["logneg"], abs=1e-9)
    assert abs(g["logneg"] - want) <= 4 * g["logneg_se"] + 1e-3


def test_quadrature_kernel_matches_oracle(dev):
    import torch
    psi = ti.haar_state(9, 1)
    o = slq.slq_logneg(psi, 9, [0, 1, 2], [5, 6, 7], 6, 30, seed=3)
    al = torch.from_numpy(o["alpha"]).to(dev)
    be = torch.from_numpy(o["beta"]).to(dev)
    F = T.tnslq_quadrature(al, be).cpu().numpy()
    assert np.allclose(F, o["F"], rtol=1e-11, atol=1e-14)


def test_stop_tolerance_stops_early_and_agrees(dev):
    import torch
    L, a, b = 14, list(range(5)), list(range(5, 10))
    psi = ti.haar_state(L, 2)
    psi_t = torch.from_numpy(psi).to(dev)
    full = T.tnslq_logneg(psi_t, L, a, b, 16, 40, precision="fp64", seed=1)
    early = T.tnslq_logneg(psi_t, L, a, b, 16, 40, precision="fp64", seed=1, stop_tol=0.01)
    assert 6 <= early["steps_done"] < 40
    assert abs(early["logneg"] - full["logneg"]) <= 0.01 * max(abs(full["logneg"]), 1.0)


@pytest.mark.parametrize("tol", [0.02, 0.01, 0.003])
def test_difference_rule_matches_oracle(dev, tol):
    # the step-difference stop (stop_rule TNSLQ_STOP_DIFF) in FP64 against
    # the oracle's rule replayed on its own trajectories for the same probes:
    # the same stop step, estimate and Lanczos proxy
    import torch
    from oracle import step_difference
    L, a, b, K, m = 14, list(range(5)), list(range(5, 10)), 16, 40
    psi = ti.haar_state(L, 2)
    g = T.tnslq_logneg(torch.from_numpy(psi).to(dev), L, a, b, K, m, precision="fp64", seed=1, stop_tol=tol,
                       stop_rule="diff", operator="lazy")
    R = exact.rho_pt(exact.regroup(psi, L, a, b))
    o = slq.slq(lambda v: R @ v, probes.rademacher_probes(1, K, 1 << 10), m)
    want = step_difference.run(o["beta"], o["F"], tol)
    # no step's error sits within rounding of its threshold, so the stop step
    # is decided the same way on both sides
    for j in range(6, want["steps"] + 1):
        c = step_difference.combined_error(o["beta"], o["F"], j)
        thr = tol * max(abs(c["logneg"]), 1.0)
        assert abs(c["err"] - thr) > 1e-9 * thr
    assert 6 <= want["steps"] < m
    assert g["steps_done"] == want["steps"]
    assert g["logneg"] == pytest.approx(want["logneg"], abs=1e-10 * max(1.0, abs(want["logneg"])))
    assert g["lanczos_err"] == pytest.approx(want["lanczos_err"], abs=1e-10)
    assert g["logneg_se"] == pytest.approx(want["logneg_se"], rel=1e-9)


def test_probe_offset_merges_as_independent_samples(dev):
    import torch
    L, a, b = 10, [0, 1, 2], [3, 4, 5]
    psi_t = torch.from_numpy(ti.haar_state(L, 0)).to(dev)
    r1 = T.tnslq_logneg(psi_t, L, a, b, 8, 10, precision="fp64", seed=5)
    r2 = T.tnslq_logneg(psi_t, L, a, b, 8, 10, precision="fp64", seed=5, probe_offset=8)
    r = T.tnslq_logneg(psi_t, L, a, b, 16, 10, precision="fp64", seed=5)
    assert np.allclose(np.concatenate([r1["G"], r2["G"]]), r["G"], rtol=1e-13, atol=0)


@pytest.mark.parametrize("operator", ["lazy", "explicit"])
def test_deterministic_rerun(dev, operator):
    import torch
    L, a, b = 12, [0, 1, 2, 3], [6, 7, 8, 9]
    psi_t = torch.from_numpy(ti.haar_state(L, 8).astype(np.complex64)).to(dev)
    r1 = T.tnslq_logneg(psi_t, L, a, b, 8, 16, precision="bf16x3", seed=1, operator=operator)
    r2 = T.tnslq_logneg(psi_t, L, a, b, 8, 16, precision="bf16x3", seed=1, operator=operator)
    assert np.array_equal(r1["alpha"], r2["alpha"]) and np.array_equal(r1["beta"], r2["beta"])
    assert r1["logneg"] == r2["logneg"]


@pytest.mark.parametrize("a,b", [(list(range(10)), [10]),            # d_B = 2: both passes 1024 columns wide
                                 ([19], list(range(3, 13)))])         # |B| > |A|: roles exchanged
@pytest.mark.parametrize("dtype", [np.complex64, np.complex128])
def test_streaming_passes_match_oracle(dev, a, b, dtype):
    # K d_B <= 8: two streaming passes over psi with FP64 arithmetic whatever
    # the precision (up to 4 vectors on the vector units, 8 on the FP64 matrix
    # instructions), so FP64-level agreement with the oracle on the same
    # (rounded) amplitudes
    import torch
    L = 20
    psi_t, psi_np = _dev_state(ti.haar_state(L, 6), dtype, dev)
    P = exact.regroup(psi_np, L, a, b)
    dab = P.shape[0] * P.shape[1]
    for K in (1, 2, 3, 4):
        X = ti.random_vectors(K, dab, seed=K + 10)
        Y = T.tnslq_ptmatvec(psi_t, L, a, b, torch.from_numpy(X).to(dev), precision="bf16x3").cpu().numpy()
        err = _relerr(Y, exact.pt_matvec_explicit(P, X))
        print(f"stream matvec a={a} b={b} K={K}: {err:.2e}")
        assert err <= 1e-12
    for K in (2, 4):
        g = T.tnslq_logneg(psi_t, L, a, b, K, 10, precision="bf16x3", seed=4, operator="lazy")
        o = slq.slq_logneg(psi_np, L, a, b, K, 10, seed=4)
        assert g["streamed"] == 1       # d_A = 1024: the two passes
        assert np.max(np.abs(g["alpha"] - o["alpha"])) <= 1e-10 * np.max(np.abs(o["alpha"]))
        assert g["logneg"] == pytest.approx(o["logneg"], abs=1e-10 * max(abs(o["logneg"]), 1.0))
