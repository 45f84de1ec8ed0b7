"""tnslq_ptmatvec_static: the block matvec on the library's fixed per-GPU
scratch (for callers that cannot allocate) gives the same result as
tnslq_ptmatvec on a caller's workspace, call after call: two calls in a row
per precision, the second on a smaller problem, each checked against the
workspace entry point and against the oracle's explicit operator."""
import numpy as np
import pytest

import tnslq_inputs as ti
from oracle import exact

pytestmark = pytest.mark.gpu
T = pytest.importorskip("paper_1809_01685_amd")

TOL = {"fp64": 1e-12, "fp32": 1e-6, "bf16x3": 3e-5}


def _case(dev, L, a, b, K, prec, seed, chunk=0):
    import torch
    dtype = np.complex128 if prec == "fp64" else np.complex64
    psi = ti.haar_state(L, seed).astype(dtype)
    n = 1 << (len(a) + len(b))
    X = ti.random_vectors(K, n, seed=seed + 100)
    psi_t = torch.from_numpy(psi).to(dev)
    Xd = torch.from_numpy(X).to(dev)
    need = T.tnslq_ptmatvec_workspace_bytes(1 if prec == "fp64" else 0, L, a, b, K, prec, chunk)
    assert need <= T.STATIC_SCRATCH_BYTES
    Ys = T.tnslq_ptmatvec_static(psi_t, L, a, b, Xd, precision=prec, chunk_vectors=chunk)
    Yw = T.tnslq_ptmatvec(psi_t, L, a, b, Xd, precision=prec, chunk_vectors=chunk)
    torch.cuda.synchronize()
    Ys, Yw = Ys.cpu().numpy(), Yw.cpu().numpy()
    ref = exact.pt_matvec_explicit(exact.regroup(psi.astype(np.complex128), L, a, b), X)
    scale = np.max(np.abs(ref))
    d_ws = float(np.max(np.abs(Ys - Yw)) / scale)
    d_or = float(np.max(np.abs(Ys - ref)) / scale)
    print(f"L={L} K={K} {prec}: vs workspace entry {d_ws:.1e} (bit-identical: {np.array_equal(Ys, Yw)}), "
          f"vs oracle {d_or:.1e}", flush=True)
    assert d_ws <= TOL[prec] and d_or <= TOL[prec]


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_static_scratch_matches_workspace_entry_point_call_after_call(dev, prec):
    # first a 14-qubit problem in chunks (the scratch holds its regrouped
    # state, probe operand and intermediary), then a smaller 12-qubit one on
    # the same scratch, whose padding is cleared afresh
    _case(dev, 14, list(range(0, 6)), list(range(8, 14)), 10, prec, seed=1, chunk=4)
    _case(dev, 12, [0, 1, 2, 3], [6, 7, 8], 3, prec, seed=2)


def test_streaming_form_on_static_scratch(dev):
    # K d_B <= 8: the two FP64 streaming passes, on the same scratch
    _case(dev, 16, list(range(0, 10)), [12], 2, "bf16x3", seed=3)
    _case(dev, 14, list(range(0, 8)), [9, 10], 1, "fp32", seed=4)
