"""Pins for the oracle's probe generator (Algorithm 1's random vectors)."""
import os

import numpy as np

from oracle import probes

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "splitmix64_seed1234567.txt")


def _golden():
    with open(GOLDEN) as f:
        return [int(line) for line in f if line.strip() and not line.startswith("#")]


def test_splitmix64_known_answer():
    want = _golden()
    got = probes.splitmix64(1234567, np.arange(len(want)))
    assert [int(x) for x in got] == want


def test_splitmix64_is_counter_based():
    # output n depends only on (seed, n): evaluating a window equals slicing a longer run
    full = probes.splitmix64(99, np.arange(1000))
    part = probes.splitmix64(99, np.arange(500, 700))
    assert np.array_equal(full[500:700], part)


def test_probe_entries_are_complex_rademacher():
    X = probes.rademacher_probes(seed=5, n_probes=8, d_ab=4096)
    allowed = np.array([1, 1j, -1, -1j])
    d = np.min(np.abs(X[..., None] - allowed[None, None, :]), axis=-1)
    assert np.all(d == 0.0)
    # every entry has unit modulus, so ||phi||^2 = d_AB exactly
    assert np.all(np.sum(np.abs(X) ** 2, axis=1) == 4096.0)
    # the four values are equally likely (binomial 5-sigma band)
    counts = np.array([np.sum(X == v) for v in allowed])
    n = X.size
    assert np.all(np.abs(counts - n / 4) < 5 * np.sqrt(n * 3 / 16))
    # zero mean and E[z^2] = 0 (circular law)
    assert abs(np.mean(X)) < 5 / np.sqrt(n)
    assert abs(np.mean(X * X)) < 5 / np.sqrt(n)


def test_probe_element_mapping_uses_top_two_bits():
    seed, d = 3, 16
    raw = probes.splitmix64(seed, np.arange(2 * d))
    r = (raw >> np.uint64(62)).astype(int)
    X = probes.rademacher_probes(seed, 2, d)
    assert np.array_equal(X.reshape(-1), np.array([1, 1j, -1, -1j])[r])


def test_probe_offset_continues_the_sequence():
    a = probes.rademacher_probes(seed=11, n_probes=5, d_ab=64)
    b = probes.rademacher_probes(seed=11, n_probes=2, d_ab=64, probe_offset=3)
    assert np.array_equal(a[3:5], b)
