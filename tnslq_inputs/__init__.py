"""Seeded synthetic inputs shared by the oracle and the GPU path.

This module holds state and partition generators only: none of the
logarithmic-negativity arithmetic (regrouping, partial transpose, Lanczos,
quadrature) lives here.  Both the CPU oracle and the HIP path take their
inputs from these functions so that they see bit-identical states.

Workloads follow the paper's experiments (Sec. VII):
  * Haar-random pure states (Sec. VII.A): i.i.d. complex Gaussian amplitudes,
    normalised in FP64.
  * A scrambling stand-in for the Heisenberg quench of Sec. VII.B: a brickwork
    circuit of Haar-random two-qubit gates applied to |0...0>.

Qubit 0 is the most significant bit of the flat amplitude index (the order of
``numpy.kron``), so a state of L qubits reshaped to ``[2]*L`` has qubit q on
axis q.
"""
from __future__ import annotations

import dataclasses
from typing import List, Sequence, Tuple

import numpy as np

__all__ = [
    "haar_state",
    "haar_state_torch",
    "haar_unitary",
    "brickwork_gates",
    "brickwork_state",
    "brickwork_state_torch",
    "basis_product_state",
    "bell_pair_state",
    "random_contiguous_partition",
    "haar_state_dims",
    "max_entangled_pair_state_dims",
    "random_mps",
    "bell_pair_mps",
    "Workload",
    "WORKLOADS",
    "random_vectors_torch",
]


# --------------------------------------------------------------------------
# Haar-random pure states (Sec. VII.A)
# --------------------------------------------------------------------------
def haar_state(n_qubits: int, seed: int, dtype=np.complex128) -> np.ndarray:
    """Haar-random pure state: Re and Im i.i.d. N(0,1), normalised in FP64.

    The amplitudes are drawn with ``numpy.random.default_rng(seed)``: first all
    real parts, then all imaginary parts.  Normalisation happens in complex128
    before any cast to ``dtype``.
    """
    n = 1 << n_qubits
    rng = np.random.default_rng(seed)
    re = rng.standard_normal(n)
    im = rng.standard_normal(n)
    psi = re + 1j * im
    psi /= np.linalg.norm(psi)
    return psi.astype(dtype, copy=False)


def haar_state_torch(n_qubits: int, seed: int, device, dtype=None):
    """Haar-random pure state generated on a torch device.

    Used for states too large to generate on the host in reasonable time
    (26 qubits and up).  The generator is torch's, seeded with ``seed``; the
    values differ from :func:`haar_state` for the same seed.  Normalisation is
    done in FP64 on the device, then the state is cast to ``dtype``.
    """
    import torch

    dtype = dtype or torch.complex64
    n = 1 << n_qubits
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    out = torch.empty(n, dtype=dtype, device=device)
    real_dtype = torch.float32 if dtype == torch.complex64 else torch.float64
    view = torch.view_as_real(out)
    chunk = 1 << 26
    norm2 = torch.zeros((), dtype=torch.float64, device=device)
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        x = torch.randn((e - s, 2), generator=g, device=device, dtype=torch.float64)
        norm2 += (x * x).sum()
        view[s:e] = x.to(real_dtype)
    scale = (1.0 / torch.sqrt(norm2)).to(real_dtype)
    view.mul_(scale)
    return out


# --------------------------------------------------------------------------
# Brickwork circuits of Haar two-qubit gates (stand-in for Sec. VII.B)
# --------------------------------------------------------------------------
def haar_unitary(n: int, rng: np.random.Generator) -> np.ndarray:
    """Haar-distributed n x n unitary (Mezzadri 2007: QR of a complex
    Ginibre matrix with the phases of R's diagonal divided out)."""
    z = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(2.0)
    q, r = np.linalg.qr(z)
    d = np.diagonal(r)
    ph = d / np.abs(d)
    return q * ph[None, :]


def brickwork_gates(n_qubits: int, depth: int, seed: int) -> List[Tuple[int, np.ndarray]]:
    """Gate list ``[(i, U), ...]`` of a brickwork circuit.

    Layer t = 1..depth acts on pairs (i, i+1) with i = t-1 (mod 2) and
    i+1 < n_qubits (open boundary).  Gates are drawn from one
    ``default_rng(seed)`` in (layer, pair) order.  Qubit i is the most
    significant bit of each 4 x 4 gate's index.
    """
    rng = np.random.default_rng(seed)
    gates = []
    for t in range(1, depth + 1):
        for i in range((t - 1) % 2, n_qubits - 1, 2):
            gates.append((i, haar_unitary(4, rng)))
    return gates


def brickwork_state(n_qubits: int, depth: int, seed: int, dtype=np.complex128) -> np.ndarray:
    """|0...0> evolved by :func:`brickwork_gates` (host, complex128)."""
    n = 1 << n_qubits
    psi = np.zeros(n, dtype=np.complex128)
    psi[0] = 1.0
    for i, u in brickwork_gates(n_qubits, depth, seed):
        v = psi.reshape(1 << i, 4, 1 << (n_qubits - i - 2))
        psi = np.einsum("ij,ajb->aib", u, v).reshape(n)
    return psi.astype(dtype, copy=False)


def brickwork_state_torch(n_qubits: int, depth: int, seed: int, device, dtype=None):
    """Same circuit as :func:`brickwork_state`, applied on a torch device.

    The gates are the host-drawn ones from :func:`brickwork_gates`; only the
    application runs on the device (in complex128, cast at the end).
    """
    import torch

    dtype = dtype or torch.complex64
    n = 1 << n_qubits
    psi = torch.zeros(n, dtype=torch.complex128, device=device)
    psi[0] = 1.0
    for i, u in brickwork_gates(n_qubits, depth, seed):
        ut = torch.from_numpy(np.ascontiguousarray(u)).to(device)
        v = psi.view(1 << i, 4, 1 << (n_qubits - i - 2))
        psi = torch.matmul(ut, v).reshape(n)
    return psi.to(dtype)


# --------------------------------------------------------------------------
# Small closed-form fixtures
# --------------------------------------------------------------------------
def basis_product_state(n_qubits: int, bits: Sequence[int], dtype=np.complex128) -> np.ndarray:
    """Computational-basis product state |bits>, bits[q] for qubit q."""
    idx = 0
    for q in range(n_qubits):
        idx = (idx << 1) | (int(bits[q]) & 1)
    psi = np.zeros(1 << n_qubits, dtype=dtype)
    psi[idx] = 1.0
    return psi


def bell_pair_state(n_qubits: int, i: int, j: int, background_seed: int | None = None,
                    dtype=np.complex128) -> np.ndarray:
    """(|00> + |11>)/sqrt(2) on qubits (i, j), every other qubit in a product
    state: |0> when ``background_seed`` is None, else a seeded random
    single-qubit state per qubit."""
    rng = np.random.default_rng(background_seed) if background_seed is not None else None
    t = np.zeros([2] * n_qubits, dtype=np.complex128)
    # Build as a tensor product over qubits other than (i, j).
    others = [q for q in range(n_qubits) if q not in (i, j)]
    singles = {}
    for q in others:
        if rng is None:
            v = np.array([1.0, 0.0], dtype=np.complex128)
        else:
            v = rng.standard_normal(2) + 1j * rng.standard_normal(2)
            v /= np.linalg.norm(v)
        singles[q] = v
    for bit in (0, 1):
        vec = np.array([1.0], dtype=np.complex128)
        for q in range(n_qubits):
            if q == i or q == j:
                e = np.zeros(2, dtype=np.complex128)
                e[bit] = 1.0
                vec = np.kron(vec, e)
            else:
                vec = np.kron(vec, singles[q])
        t += vec.reshape([2] * n_qubits) / np.sqrt(2.0)
    return t.reshape(-1).astype(dtype, copy=False)


# --------------------------------------------------------------------------
# Partitions
# --------------------------------------------------------------------------
def random_contiguous_partition(n_qubits: int, rng: np.random.Generator) -> Tuple[List[int], List[int]]:
    """Contiguous blocks A then B (|A|, |B| >= 1, gap >= 0) at a random
    offset, as used for the surrogate's training instances."""
    while True:
        na = int(rng.integers(1, n_qubits))
        nb = int(rng.integers(1, n_qubits))
        gap = int(rng.integers(0, n_qubits))
        span = na + gap + nb
        if span <= n_qubits:
            break
    start = int(rng.integers(0, n_qubits - span + 1))
    a = list(range(start, start + na))
    b = list(range(start + na + gap, start + na + gap + nb))
    return a, b


@dataclasses.dataclass(frozen=True)
class Workload:
    """A named workload: state recipe, partition and SLQ sizes."""
    name: str
    n_qubits: int
    a: Tuple[int, ...]
    b: Tuple[int, ...]
    n_probes: int
    n_steps: int
    state: str            # "haar" or "brickwork"
    dtype: str            # "c64" or "c128"
    precision: str        # "fp64", "fp32", "bf16x3", "bf16x6"
    reorth: bool
    depth: int = 0

    @property
    def e(self) -> Tuple[int, ...]:
        s = set(self.a) | set(self.b)
        return tuple(q for q in range(self.n_qubits) if q not in s)


WORKLOADS = {
    # 10-qubit Haar state, A = 0-2, B = 3-5, E = 6-9; exact 64 x 64 eigensolve
    # against SLQ with 16 probes and 20 steps.
    "haar10": Workload("haar10", 10, (0, 1, 2), (3, 4, 5), 16, 20, "haar", "c128", "fp64", False),
    # 20-qubit Haar state, |A| = |B| = 6 separated by 2 qubits, E = 8 qubits;
    # 32 probes, 40 steps, full reorthogonalisation.
    "haar20": Workload("haar20", 20, tuple(range(0, 6)), tuple(range(8, 14)), 32, 40, "haar", "c64",
                       "fp32", True),
    # 30-qubit Haar state in complex64 (8 GiB), E = 0-3, A = 4-16, B = 17-29:
    # a 26-qubit rho_AB; 8 probes, 50 steps, split-BF16 contractions.
    "haar30": Workload("haar30", 30, tuple(range(4, 17)), tuple(range(17, 30)), 8, 50, "haar", "c64",
                       "bf16x3", False),
    # 24-qubit brickwork state, A = 4-11, B = 13-20, E = rest; 32 probes,
    # 40 steps, split-BF16.
    "brick24": Workload("brick24", 24, tuple(range(4, 12)), tuple(range(13, 21)), 32, 40, "brickwork",
                        "c64", "bf16x3", True, depth=12),
}


# --------------------------------------------------------------------------
# Surrogate network initial weights
# --------------------------------------------------------------------------
MLP_SHAPES = [((256, 19), True), ((256,), False), ((256, 256), True), ((256,), False),
              ((2, 256), True), ((2,), False)]


def mlp_init_params(seed: int) -> np.ndarray:
    """Flat float32 initial parameters of the 19-256-256-2 surrogate network
    (W1, b1, W2, b2, W3, b3): He-uniform weights from ``default_rng(seed)``,
    zero biases."""
    rng = np.random.default_rng(seed)
    parts = []
    for shape, is_weight in MLP_SHAPES:
        if is_weight:
            lim = np.sqrt(6.0 / shape[1])
            parts.append(rng.uniform(-lim, lim, size=shape).reshape(-1))
        else:
            parts.append(np.zeros(shape))
    return np.concatenate(parts).astype(np.float32)


def random_vectors(n_vectors: int, dim: int, seed: int) -> np.ndarray:
    """(n_vectors, dim) complex128 vectors with i.i.d. N(0,1) real and
    imaginary parts, from ``default_rng(seed)``."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((n_vectors, dim)) + 1j * rng.standard_normal((n_vectors, dim))


def random_vectors_torch(n_vectors: int, dim: int, seed: int, device):
    """(n_vectors, dim) complex128 vectors with i.i.d. N(0,1) real and
    imaginary parts drawn on a torch device (for blocks too large to draw on
    the host quickly), torch's generator seeded with ``seed``."""
    import torch

    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    out = torch.empty((n_vectors, dim), dtype=torch.complex128, device=device)
    torch.view_as_real(out).normal_(generator=g)
    return out


# --------------------------------------------------------------------------
# Sites of any local dimension (site 0 most significant in the flat index)
# --------------------------------------------------------------------------
def haar_state_dims(dims: Sequence[int], seed: int, dtype=np.complex128) -> np.ndarray:
    """Haar-random pure state on sites with dims[s] levels each."""
    rng = np.random.default_rng(seed)
    n = int(np.prod(list(dims), dtype=np.int64))
    v = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    v /= np.linalg.norm(v)
    return v.astype(dtype)


def max_entangled_pair_state_dims(dims: Sequence[int], i: int, j: int, dtype=np.complex128) -> np.ndarray:
    """(1/sqrt d) sum_k |k>_i |k>_j on sites i, j (d = dims[i] = dims[j]),
    every other site in level 0."""
    dims = list(dims)
    d = dims[i]
    if dims[j] != d:
        raise ValueError("the two sites need the same dimension")
    t = np.zeros(dims, dtype=np.complex128)
    for k in range(d):
        idx = [0] * len(dims)
        idx[i] = idx[j] = k
        t[tuple(idx)] = 1.0 / np.sqrt(d)
    return t.reshape(-1).astype(dtype)


# --------------------------------------------------------------------------
# Matrix product states (Sec. VI): tensors (chi_i, p, chi_{i+1}); open
# boundaries have chi_0 = chi_L = 1, periodic ones chi_0 = chi_L > 1
# --------------------------------------------------------------------------
def random_mps(n_sites: int, p: int, chi: int, seed: int) -> List[np.ndarray]:
    """Complex Gaussian tensors with bond dimensions min(chi, p^i, p^(L-i))
    (the largest an open chain can use), not normalised."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n_sites):
        cl = min(chi, p ** i, p ** (n_sites - i))
        cr = min(chi, p ** (i + 1), p ** (n_sites - i - 1))
        out.append(rng.standard_normal((cl, p, cr)) + 1j * rng.standard_normal((cl, p, cr)))
    return out


def bell_pair_mps(n_sites: int, i: int, j: int) -> List[np.ndarray]:
    """(|00> + |11>)/sqrt 2 on qubits i < j, |0> elsewhere, as an MPS of bond
    dimension 2 between i and j (1 elsewhere)."""
    out = []
    for s in range(n_sites):
        inside = i < s < j
        cl = 2 if i < s <= j else 1
        cr = 2 if i <= s < j else 1
        M = np.zeros((cl, 2, cr), dtype=np.complex128)
        if s == i:
            M[0, 0, 0] = M[0, 1, 1] = 2 ** -0.5
        elif s == j:
            M[0, 0, 0] = M[1, 1, 0] = 1.0
        elif inside:
            M[0, 0, 0] = M[1, 0, 1] = 1.0
        else:
            M[0, 0, 0] = 1.0
        out.append(M)
    return out


def random_mps_periodic(n_sites: int, p: int, chi: int, seed: int) -> List[np.ndarray]:
    """Complex Gaussian tensors of a ring: every bond chi, the closing bond
    included, not normalised."""
    rng = np.random.default_rng(seed)
    return [rng.standard_normal((chi, p, chi)) + 1j * rng.standard_normal((chi, p, chi)) for _ in range(n_sites)]


def dimer_mps(n_sites: int, seed: int, offset: int = 0, periodic: bool = False):
    """Qubit pairs (i, i+1) for i = offset, offset + 2, ... each in a random
    pure two-qubit state c[s][t] (complex Gaussian, normalised); on a ring
    (periodic) with an odd offset and an even n_sites the last pair closes
    through the boundary, (n_sites - 1, 0).  Unpaired sites are |0>.  Returns
    (tensors, pairs) with pairs a list of ((i, j), c).  Bond 2 inside a pair,
    1 elsewhere."""
    rng = np.random.default_rng(seed)
    L = n_sites
    pairs = []
    i = offset % 2
    while i + 1 < L:
        pairs.append((i, i + 1))
        i += 2
    if periodic and i == L - 1 and offset % 2 == 1:
        pairs.append((L - 1, 0))
    coef = []
    for _ in pairs:
        c = rng.standard_normal((2, 2)) + 1j * rng.standard_normal((2, 2))
        coef.append(c / np.linalg.norm(c))
    first = {a: k for k, (a, _) in enumerate(pairs)}
    second = {b: k for k, (_, b) in enumerate(pairs)}
    bond = [1] * (L + 1)
    for a, b in pairs:
        if b == a + 1:
            bond[a + 1] = 2
        else:                      # the pair closing the ring
            bond[0] = bond[L] = 2
    out = []
    for s in range(L):
        M = np.zeros((bond[s], 2, bond[s + 1]), dtype=np.complex128)
        if s in first:             # M[0][s][k] = c[s][k], the bond carries the partner's level
            M[0, :, :] = coef[first[s]]
        elif s in second:          # M[k][t][0] = delta(k, t)
            M[0, 0, 0] = M[1, 1, 0] = 1.0
        else:
            M[0, 0, 0] = 1.0
        out.append(M)
    return out, [(pr, c) for pr, c in zip(pairs, coef)]


def ghz_mps(n_sites: int, periodic: bool = True) -> List[np.ndarray]:
    """(|0...0> + |1...1>) (not normalised) as bond-2 tensors: on a ring every
    M[:, s, :] = |s><s|, so psi = Tr prod = [all s equal]; open boundaries cut
    the first and last tensors to a row and a column of ones."""
    out = []
    for s in range(n_sites):
        M = np.zeros((2, 2, 2), dtype=np.complex128)
        M[0, 0, 0] = M[1, 1, 1] = 1.0
        if not periodic and s == 0:
            M = M.sum(axis=0, keepdims=True)
        if not periodic and s == n_sites - 1:
            M = M.sum(axis=2, keepdims=True)
        out.append(M)
    return out
