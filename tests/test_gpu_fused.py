"""The one-read streaming matvec (Sec. V, Eq. 4, intermediary (i)): in the
HBM-bound regime (one vector, d_B = 2, d_A = 2048 or 4096) each block
finishes one environment slab at a time and keeps its share of Y on chip, so
psi is read once per matvec.  Against the oracle, FP64-exact: every output
entry of block matvecs over the shapes it serves (both instances, roles
exchanged, scattered partitions), and the Lanczos coefficients of whole
estimates; against the two-pass form of the same matvec, and rerun for
bitwise determinism."""
import numpy as np
import pytest

import tnslq_inputs as ti
from oracle import exact, slq

pytestmark = pytest.mark.gpu
T = pytest.importorskip("paper_1809_01685_amd")

CASES = [
    # L, A, B, K: device roles (d_A, d_B) after the exchange of roles if any
    (20, list(range(0, 11)), [11], 1),            # (2048, 2)
    (20, list(range(9, 20)), [4], 1),             # (2048, 2), E at the front
    (20, [19], list(range(3, 14)), 1),            # exchanged: (2048, 2)
    (21, list(range(0, 12)), [15], 1),            # (4096, 2), B inside E
    (21, [0, 2, 4, 6, 8, 10, 12, 14, 16, 18, 20, 1], [3], 1),   # (4096, 2), scattered
    (22, list(range(4, 16)), [17], 1),            # (4096, 2), 1024 slabs
]


def _run(dev, L, a, b, K, operator=None):
    import torch
    psi = ti.haar_state(L, L + K).astype(np.complex64)
    n = 1 << (len(a) + len(b))
    X = ti.random_vectors(K, n, seed=L * 7 + K)
    psi_t = torch.from_numpy(psi).to(dev)
    Y = T.tnslq_ptmatvec(psi_t, L, a, b, torch.from_numpy(X).to(dev), precision="bf16x3").cpu().numpy()
    return psi, X, Y


@pytest.mark.parametrize("L,a,b,K", CASES)
def test_one_read_matvec_matches_oracle_entrywise(dev, L, a, b, K):
    psi, X, Y = _run(dev, L, a, b, K)
    P = exact.regroup(psi.astype(np.complex128), L, a, b)
    ref = exact.pt_matvec_explicit(P, X) if P.shape[0] * P.shape[1] <= 4096 else exact.pt_matvec_lazy(P, X)
    err = float(np.max(np.abs(Y - ref)) / np.max(np.abs(ref)))
    print(f"L={L} |A|={len(a)} |B|={len(b)} K={K}: max error / max |Y| = {err:.1e}")
    assert err <= 1e-12


@pytest.mark.parametrize("L,a,b,K", [CASES[0], CASES[2], CASES[3], CASES[5]])
def test_one_read_estimate_matches_oracle_and_two_pass(dev, L, a, b, K):
    # alpha, beta and E of an FP64 estimate (the streaming regime runs FP64
    # whatever the requested precision) on the same probes; the two-pass form
    # gives the same coefficients to rounding, and a rerun the same bits
    import torch
    psi = ti.haar_state(L, 3).astype(np.complex64)
    psi_t = torch.from_numpy(psi).to(dev)
    m = 10
    g = T.tnslq_logneg(psi_t, L, a, b, K, m, precision="bf16x3", seed=5, operator="lazy")
    g2 = T.tnslq_logneg(psi_t, L, a, b, K, m, precision="bf16x3", seed=5, operator="lazy_two_pass")
    g3 = T.tnslq_logneg(psi_t, L, a, b, K, m, precision="bf16x3", seed=5, operator="lazy")
    assert g["streamed"] == 2 and g2["streamed"] == 1
    assert np.array_equal(g["alpha"], g3["alpha"]) and np.array_equal(g["beta"], g3["beta"])
    scale = np.max(np.abs(g2["alpha"]))
    assert np.max(np.abs(g["alpha"] - g2["alpha"])) <= 1e-11 * scale
    if (1 << (len(a) + len(b))) <= 4096:
        o = slq.slq_logneg(psi.astype(np.complex128), L, a, b, K, m, seed=5)
        assert np.max(np.abs(g["alpha"] - o["alpha"])) <= 1e-10 * np.max(np.abs(o["alpha"]))
        assert g["logneg"] == pytest.approx(o["logneg"], abs=1e-10 * max(1.0, abs(o["logneg"])))
