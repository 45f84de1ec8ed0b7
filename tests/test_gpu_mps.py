"""GPU parity of the matrix-product-state reduction (Sec. VI) against the
oracle, through the C ABI.

The effective state is unique (Cholesky factors with a positive diagonal), so
the device's matches the oracle's entry by entry: 1e-11 of its largest entry
(FP64 products over sections of up to 2^7 physical values and Cholesky
factors of matrices up to 256 wide).  Its padding holds zeros.  The estimate
then runs through tnslq_logneg on the padded state; in FP64 its Lanczos
coefficients match the oracle's on the same padded state and probes to 1e-10.
"""
import numpy as np
import pytest

import tnslq_inputs as ti
from oracle import exact, mps, slq

pytestmark = pytest.mark.gpu

T = pytest.importorskip("paper_1809_01685_amd")

GEOMETRIES = [
    (12, 4, 2, 4, 6, 4),     # adjacent blocks
    (12, 4, 2, 4, 8, 3),     # gap of 2 sites, not compressed
    (12, 3, 0, 5, 5, 7),     # A at the left end, B at the right end, both compressed
    (14, 4, 1, 5, 8, 6),     # B at the right end, gap 2
    (14, 2, 1, 3, 9, 3),     # gap of 5 sites compressed
    (10, 8, 1, 3, 5, 3),
    (16, 4, 3, 7, 11, 4),    # A compressed (2^7 > 16), gap 1
]


def _padded(Pe, q):
    dA, dB, dE = Pe.shape
    out = np.zeros((1 << q[0], 1 << q[1], 1 << q[2]), dtype=np.complex128)
    out[:dA, :dB, :dE] = Pe
    return out


@pytest.mark.parametrize("L,chi,a0,LA,b0,LB", GEOMETRIES)
def test_effective_state_matches_oracle(dev, L, chi, a0, LA, b0, LB):
    ts = ti.random_mps(L, 2, chi, L + chi)
    psi, q = T.tnslq_mps_effective_state(ts, a0, LA, b0, LB, device=dev)
    Pe = mps.effective_state(ts, a0, LA, b0, LB)
    want = _padded(Pe, q)
    got = psi.cpu().numpy().reshape(want.shape)
    assert np.max(np.abs(got - want)) <= 1e-11 * np.max(np.abs(want))


@pytest.mark.parametrize("L,chi,a0,LA,b0,LB", [GEOMETRIES[0], GEOMETRIES[3], GEOMETRIES[6]])
def test_logneg_of_blocks_matches_oracle(dev, L, chi, a0, LA, b0, LB):
    ts = ti.random_mps(L, 2, chi, L + chi)
    g = T.tnslq_logneg_mps(ts, a0, LA, b0, LB, 8, 16, device=dev, precision="fp64", seed=2, reorth=True)
    qa, qb, qe = g["effective_qubits"]
    Pp = _padded(mps.effective_state(ts, a0, LA, b0, LB), (qa, qb, qe))
    o = slq.slq_logneg(Pp.reshape(-1), qa + qb + qe, list(range(qa)), list(range(qa, qa + qb)), 8, 16, seed=2,
                       reorth=True)
    assert np.max(np.abs(g["alpha"] - o["alpha"])) <= 1e-10 * np.max(np.abs(o["alpha"]))
    assert g["logneg"] == pytest.approx(o["logneg"], abs=1e-10 * max(abs(o["logneg"]), 1.0))
    # and the estimate against the exact value of the whole chain's blocks
    psi = mps.mps_to_dense(ts)
    e = exact.logneg_exact(exact.regroup(psi / np.linalg.norm(psi), L, list(range(a0, a0 + LA)),
                                         list(range(b0, b0 + LB))))
    assert abs(g["logneg"] - e) <= 4 * g["logneg_se"] + 0.02 * max(abs(e), 1.0)


def test_bell_pair_blocks_give_one_bit(dev):
    ts = ti.bell_pair_mps(12, 2, 9)
    r = T.tnslq_logneg_mps(ts, 1, 3, 7, 4, 4, 10, device=dev, precision="fp64", seed=0)
    assert r["logneg"] == pytest.approx(1.0, abs=1e-12)
