"""Hutchinson probe vectors (Sec. III, Algorithm 1: a zero-mean, unit-variance
random vector per repeat).

Oracle, test infrastructure only.

Probe law: complex Rademacher, phi[i] = 1j**r with r uniform on {0,1,2,3}.
It has E[z] = E[z^2] = 0 and |z| = 1, so ||phi||^2 = d_A d_B exactly.

Random bits: SplitMix64 (Steele, Lea & Flood, OOPSLA 2014), in the form of
Vigna's public reference generator: state x advances by the golden-gamma
0x9E3779B97F4A7C15 and each output is the avalanche mix of the new state.
Its n-th output (n = 0, 1, ...) for seed s is therefore mix(s + (n+1)*gamma),
which makes it counter-based.  Probe k (counting from ``probe_offset``),
element i = a*d_B + b (a over A's qubits, b over B's, each in the order the
partition lists them, first qubit most significant) uses counter
n = (probe_offset + k) * d_A * d_B + i, and r is the top two bits of the
output.
"""
from __future__ import annotations

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
MIX1 = np.uint64(0xBF58476D1CE4E5B9)
MIX2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, counters: np.ndarray) -> np.ndarray:
    """Outputs number ``counters`` (0-based) of SplitMix64 seeded with ``seed``."""
    n = np.asarray(counters, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + (n + np.uint64(1)) * GAMMA
        z = (z ^ (z >> np.uint64(30))) * MIX1
        z = (z ^ (z >> np.uint64(27))) * MIX2
        z = z ^ (z >> np.uint64(31))
    return z


def rademacher_probes(seed: int, n_probes: int, d_ab: int, probe_offset: int = 0) -> np.ndarray:
    """(n_probes, d_ab) complex128 probes with entries in {1, 1j, -1, -1j}."""
    k = np.arange(n_probes, dtype=np.uint64)[:, None] + np.uint64(probe_offset)
    i = np.arange(d_ab, dtype=np.uint64)[None, :]
    r = (splitmix64(seed, k * np.uint64(d_ab) + i) >> np.uint64(62)).astype(np.int64)
    table = np.array([1.0 + 0.0j, 0.0 + 1.0j, -1.0 + 0.0j, 0.0 - 1.0j])
    return table[r]
