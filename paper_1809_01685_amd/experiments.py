"""Experiment drivers on the library (the paper's Sec. VII set-ups, adapted).

    python -m paper_1809_01685_amd.experiments scrambling [--depths 1-12]
        24-qubit brickwork states of Haar two-qubit gates from |0...0>, A = 4-11,
        B = 13-20, E = rest: logarithmic negativity against circuit depth
        (a seeded stand-in for the quench of Sec. VII.B).

    python -m paper_1809_01685_amd.experiments heldout26 [--models DIR,...]
        The early-stopping surrogate on 26-qubit rho_AB it never saw: the
        30-qubit Haar state (E = 0-3) and 28-qubit brickwork states (A = 1-13,
        B = 14-26, E = {0, 27}) at depths 4, 8, 12.  Each is judged against
        50-step split-BF16 SLQ on the same probes, beside the +-1% stop of the
        exponential-fit rule, with the time of each.

    python -m paper_1809_01685_amd.experiments rounding [--depth 8]
        How far plain (not reorthogonalised) Lanczos moves with the matvec's
        rounding: one 28-qubit brickwork state of the held-out set, the same 8
        probes in split BF16 and in FP32, after 12 and after 50 steps.

    python -m paper_1809_01685_amd.experiments surrogate_latency [--model DIR]
        The learned stop's inference latency: the network on one feature row,
        and the whole decision inside the surrogate run on a 20-qubit state.

    python -m paper_1809_01685_amd.experiments entropy30
        Von Neumann entropy of the 30-qubit Haar state (complex64) for cuts of
        15 and 13 qubits and 4-16 probes, against Page's value, with the time
        per Lanczos step and the HBM throughput of the two streaming passes
        over psi that apply the reduced density matrix.

    python -m paper_1809_01685_amd.experiments hbm_sweep [--cases 13:1:1,...]
        The HBM-bound end of the negativity: the 30-qubit Haar state with
        A = 4.. (|A| = 10, 12, 13 qubits) and B the next 1-3 qubits, K = 1, 2, 4
        probes, 10 Lanczos steps, in the one-read form where the shape has it
        and in the two-pass form; time per block matvec against the minimum
        bytes (psi once, the probe block in and out) at 8 TB/s.

    python -m paper_1809_01685_amd.experiments operator_forms
        The lazy operator (intermediary (i)) against the explicit one
        (intermediary (iii)) on Haar states where d_A d_B <= 16384: 10 qubits
        (d_A d_B = 64), the 20-qubit workload (4096, d_E = 256, K = 32, 40
        steps with reorthogonalisation) in three precisions, and 24 qubits
        with A = 0-6, B = 7-13 (16384, d_E = 1024); wall time per estimate,
        and which form the automatic choice takes.

    python -m paper_1809_01685_amd.experiments hbm_peak
        What HBM bandwidth is reachable on this GPU, as a yardstick for the
        streaming passes: torch's device-to-device copy of 4 GiB and its sum
        over 8 GiB of float32 (vendor kernels, timed with events), beside the
        entropy passes over the 30-qubit state (8 GiB, complex64) at K = 1, 2, 4.

    python -m paper_1809_01685_amd.experiments mps_blocks
        Two contiguous blocks of a 100-site random open-boundary MPS (qubits,
        complex Gaussian tensors, bond dimension chi): adjacent 16-site blocks
        at chi = 16 and 32 (the geometry of Sec. VII.C), 8-site blocks at
        chi = 64 and 180 (the paper's largest bond dimension), and blocks 1 or
        4 sites apart; the dense route (effective
        state, then the split-BF16 estimate) against the factorised operator
        (FP64), both to +-1% by the exponential-fit rule.

    python -m paper_1809_01685_amd.experiments mps_long
        Long blocks at the size of Sec. VII.C's Heisenberg chain: a 1000-site
        random open MPS with bond 32, 64 and 116, adjacent blocks of 20, 100
        and 400 sites at its centre (their Gram matrices from transfer
        sweeps), the factorised operator in FP32 to +-1% by the fit rule;
        80-site blocks 40 sites apart (bond 16: both matvec forms; bond 64:
        the network form); then rings of 200 sites, bond 8 to 32, blocks of
        40 sites 10 apart and a 110-site outer section.

    python -m paper_1809_01685_amd.experiments arith_peaks
        Achievable arithmetic rates of this GPU (libtnslq_peak): dependent
        loops of the BF16, FP32 and FP64 matrix instructions the contractions
        use, and of FP64 and FP32 vector FMAs, each over 2048 workgroups of
        four waves with eight (sixteen) independent chains per wave; best and
        median of 5 launches of about 50 ms, against the published peaks.

All print one JSON object.  All arithmetic of the method runs in libtnslq
(hbm_peak times torch's own copy and sum only as a reference).
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np

from . import MLP_NIN, tnslq_logneg


def _trajectory(r):
    """E_j and its error on the mean for every step j of a run."""
    G = r["beta"][:, :1] ** 2 * r["F"][:, :r["steps_done"]]
    mean = G.mean(axis=0)
    K = G.shape[0]
    se = G.std(axis=0, ddof=1) / math.sqrt(K) if K > 1 else np.full(mean.shape, np.nan)
    return np.log2(mean), se / (mean * math.log(2.0))


def _adaptive_stop(E, dE, tol=0.01):
    """First step j >= 6 with sqrt(dE_j^2 + (E_j - E_{j-5})^2) <= tol max(|E_j|, 1)."""
    for j in range(6, len(E) + 1):
        err = math.sqrt((0.0 if np.isnan(dE[j - 1]) else dE[j - 1] ** 2) + (E[j - 1] - E[j - 6]) ** 2)
        if err <= tol * max(abs(E[j - 1]), 1.0):
            return j
    return len(E)


def run_scrambling(depths, seed=0, n_probes=32, n_steps=40, precision="bf16x3"):
    import torch
    import tnslq_inputs as ti
    w = ti.WORKLOADS["brick24"]
    dev = torch.device("cuda:0")
    rows = []
    for depth in depths:
        psi = ti.brickwork_state_torch(w.n_qubits, depth, seed, dev, torch.complex64)
        t0 = time.perf_counter()
        r = tnslq_logneg(psi, w.n_qubits, list(w.a), list(w.b), n_probes, n_steps, reorth=w.reorth,
                         precision=precision, seed=seed)
        sec = time.perf_counter() - t0
        # the same probes under the fit rule without a target: the fitted
        # limit at the last step and the fit's Lanczos error
        f = tnslq_logneg(psi, w.n_qubits, list(w.a), list(w.b), n_probes, n_steps, reorth=w.reorth,
                         precision=precision, seed=seed, stop_rule="fit", want_arrays=False)
        rows.append({"depth": depth, "logneg": r["logneg"], "logneg_se": r["logneg_se"],
                     "lanczos_err_step_difference": r["lanczos_err"], "logneg_fit": f["logneg"],
                     "lanczos_err_fit": f["lanczos_err"], "steps_min": r["steps_min"], "seconds": sec})
        print(f"[scrambling] depth {depth}: E = {r['logneg']:.4f} +- {r['logneg_se']:.4f} (Hutchinson), "
              f"|E_40 - E_35| = {r['lanczos_err']:.4f}, fit {f['logneg']:.4f} +- {f['lanczos_err']:.4f} (Lanczos)",
              file=sys.stderr, flush=True)
    return {"workload": "brick24: 24-qubit brickwork, A = 4-11, B = 13-20", "probes": n_probes, "steps": n_steps,
            "precision": precision, "rows": rows}


def run_surrogate_latency(reps=200, model_dir=None):
    """Inference latency of the learned stop: the network on one feature row
    (device time between events, and host time of a forward plus a
    synchronisation), and the whole decision inside tnslq_logneg_surrogate
    (features, network, read-back) as the difference against tnslq_logneg
    running the same early steps, on a 20-qubit state."""
    import torch
    import tnslq_inputs as ti
    from . import tnslq_mlp_forward
    from .surrogate import Model, surrogate_logneg
    dev = torch.device("cuda:0")
    model = Model.load(model_dir) if model_dir else Model.load()
    p, nd = model.device_tensors(dev)
    x = torch.randn(1, MLP_NIN, dtype=torch.float32, device=dev)
    ws = torch.empty(1 << 20, dtype=torch.uint8, device=dev)
    for _ in range(10):
        tnslq_mlp_forward(p, nd, x, workspace=ws)
    torch.cuda.synchronize()
    st = torch.cuda.current_stream(dev)
    dev_us, host_us = [], []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record(st)
        tnslq_mlp_forward(p, nd, x, workspace=ws)
        e1.record(st)
        torch.cuda.synchronize()
        host_us.append((time.perf_counter() - t0) * 1e6)
        dev_us.append(e0.elapsed_time(e1) * 1e3)
    L, a, b, K = 20, list(range(2, 11)), list(range(11, 20)), 8
    psi = ti.haar_state_torch(L, 3, dev, torch.complex64)
    n_early = model.feature_steps
    t_plain, t_sur = [], []
    for _ in range(12):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        tnslq_logneg(psi, L, a, b, K, n_early, precision="bf16x3", seed=1, want_arrays=False)
        t_plain.append(time.perf_counter() - t0)
        t0 = time.perf_counter()
        r = surrogate_logneg(model, psi, L, a, b, K, 40, tol=1e9, precision="bf16x3", seed=1)
        t_sur.append(time.perf_counter() - t0)
        assert not r["used_fallback"] and r["steps_done"] == n_early
    t_plain, t_sur = np.median(t_plain[2:]), np.median(t_sur[2:])
    out = {"n_early": n_early, "forward_device_us_median": float(np.median(dev_us)),
           "forward_host_us_median": float(np.median(host_us)),
           "decision_state": "20-qubit Haar, A = 2-10, B = 11-19, K = 8, split BF16",
           "t_plain_early_steps_ms": 1e3 * float(t_plain), "t_surrogate_accepted_ms": 1e3 * float(t_sur),
           "decision_overhead_ms": 1e3 * float(t_sur - t_plain)}
    print(f"[surrogate_latency] forward {out['forward_device_us_median']:.1f} us on the device, "
          f"{out['forward_host_us_median']:.1f} us with the synchronisation; decision overhead "
          f"{out['decision_overhead_ms']:.3f} ms", file=sys.stderr, flush=True)
    return out


def run_heldout26(n_probes=8, n_steps=50, precision="bf16x3", seed=0, tol=0.01, models=None):
    """The surrogate on rho_AB of 26 qubits it never saw, against the
    exponential-fit stop at the same target and 50-step SLQ on the same
    probes; `models` are checkpoint directories (default: the committed
    one)."""
    import torch
    import tnslq_inputs as ti
    from .surrogate import Model, surrogate_logneg
    dev = torch.device("cuda:0")
    models = models or [None]
    loaded = [(m or "committed", Model.load(m) if m else Model.load()) for m in models]
    cases = [("haar30", 30, list(range(4, 17)), list(range(17, 30)), "haar", 0)]
    for depth in (4, 8, 12):
        cases.append((f"brick28_d{depth}", 28, list(range(1, 14)), list(range(14, 27)), "brickwork", depth))
    rows = []
    for name, L, a, b, kind, depth in cases:
        if kind == "haar":
            psi = ti.haar_state_torch(L, seed, dev, torch.complex64)
        else:
            psi = ti.brickwork_state_torch(L, depth, seed, dev, torch.complex64)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        full = tnslq_logneg(psi, L, a, b, n_probes, n_steps, precision=precision, seed=seed, want_arrays=False)
        t_full = time.perf_counter() - t0
        ref = full["logneg"]
        t0 = time.perf_counter()
        fit = tnslq_logneg(psi, L, a, b, n_probes, n_steps, precision=precision, seed=seed, stop_tol=tol,
                           stop_rule="fit", want_arrays=False)
        t_fit = time.perf_counter() - t0
        row = {"case": name, "E_full": ref, "E_full_se": full["logneg_se"], "t_full_s": t_full,
               "steps_full": full["steps_done"], "fit_steps": fit["steps_done"], "E_fit": fit["logneg"],
               "err_fit": fit["logneg"] - ref, "fit_lanczos_err": fit["lanczos_err"], "t_fit_s": t_fit,
               "surrogates": []}
        for label, model in loaded:
            t0 = time.perf_counter()
            s = surrogate_logneg(model, psi, L, a, b, n_probes, n_steps, tol=tol, precision=precision, seed=seed,
                                 stop_tol=tol, stop_rule="fit")
            t_sur = time.perf_counter() - t0
            row["surrogates"].append({"model": label, "n_early": model.feature_steps, "mu": s["mu"],
                                      "sigma": s["sigma"], "accepted": not s["used_fallback"],
                                      "steps": s["steps_done"], "E_surrogate": s["logneg"],
                                      "err_surrogate": s["logneg"] - ref, "t_surrogate_s": t_sur})
            print(f"[heldout26] {name} ({label}, {model.feature_steps} steps): surrogate {s['logneg']:.5f} "
                  f"(sigma {s['sigma']:.4f}, accepted {not s['used_fallback']}, {s['steps_done']} steps, "
                  f"{t_sur:.2f} s)", file=sys.stderr, flush=True)
        rows.append(row)
        print(f"[heldout26] {name}: full {ref:.5f} ({t_full:.2f} s), fit rule {fit['logneg']:.5f} at step "
              f"{fit['steps_done']} ({t_fit:.2f} s)", file=sys.stderr, flush=True)
        del psi
        torch.cuda.empty_cache()
    return {"probes": n_probes, "steps": n_steps, "precision": precision, "tol": tol, "rows": rows}


def run_rounding(depth=8, seed=0, n_probes=8, steps=(12, 50), precisions=("bf16x3", "fp32")):
    """The held-out brickwork state (28 qubits, A = 1-13, B = 14-26) through
    the library in two precisions on the same probes, without
    reorthogonalisation: the estimates agree while Lanczos keeps its basis
    orthogonal and drift apart once it loses it (Algorithm 1 run as written)."""
    import torch
    import tnslq_inputs as ti
    dev = torch.device("cuda:0")
    L, a, b = 28, list(range(1, 14)), list(range(14, 27))
    psi = ti.brickwork_state_torch(L, depth, seed, dev, torch.complex64)
    rows = []
    for m in steps:
        for prec in precisions:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = tnslq_logneg(psi, L, a, b, n_probes, m, precision=prec, seed=seed, want_arrays=False)
            t = time.perf_counter() - t0
            rows.append({"steps": m, "precision": prec, "logneg": r["logneg"], "logneg_se": r["logneg_se"],
                         "seconds": t})
            print(f"[rounding] depth {depth}, {m} steps, {prec}: E = {r['logneg']:.6f} +- {r['logneg_se']:.4f} "
                  f"({t:.1f} s)", file=sys.stderr, flush=True)
    return {"workload": f"brick28_d{depth}: 28-qubit brickwork, A = 1-13, B = 14-26, {n_probes} probes, "
                        "no reorthogonalisation", "rows": rows}


def run_entropy30(n_steps=20, seed=0):
    import torch
    import tnslq_inputs as ti
    from . import tnslq_spectral_sum
    dev = torch.device("cuda:0")
    L = 30
    psi = ti.haar_state_torch(L, seed, dev, torch.complex64)
    esz = 8
    rows = []
    for n_s, K in ((15, 4), (15, 8), (15, 16), (13, 8)):
        s = list(range(n_s))
        tnslq_spectral_sum(psi, L, s, "entropy", K, 2, seed=seed, want_arrays=False)   # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = tnslq_spectral_sum(psi, L, s, "entropy", K, n_steps, seed=seed, want_arrays=False)
        wall = time.perf_counter() - t0
        d, dr = 1 << min(n_s, L - n_s), 1 << max(n_s, L - n_s)
        # Page's mean entropy (d <= d_R), the harmonic sum by digamma-free
        # differences of logs plus the Euler-Maclaurin terms
        n1, n2 = d * dr, dr
        harm = math.log(n1 / n2) + 0.5 / n1 - 0.5 / n2 - 1.0 / (12 * n1 * n1) + 1.0 / (12 * n2 * n2)
        page = (harm - (d - 1) / (2.0 * dr)) / math.log(2.0)
        ms_step = r["t_matvec_ms"] / n_steps
        # algorithmic bytes of one step's two passes: psi read twice, plus the
        # vectors (K d and K d_R FP64 complex, each read and written once)
        step_bytes = 2 * esz * (1 << L) + 2 * 16 * K * (d + dr)
        rows.append({"subsystem_qubits": n_s, "probes": K, "steps": n_steps, "entropy": r["value"],
                     "entropy_se": r["value_se"], "page": page, "error_vs_page": r["value"] - page,
                     "matvec_ms_per_step": ms_step, "lanczos_ms_per_step": r["t_lanczos_ms"] / n_steps,
                     "layout_ms": r["t_layout_ms"], "wall_s": wall,
                     "hbm_GBps_matvec": step_bytes / (ms_step * 1e-3) / 1e9,
                     "hbm_frac_of_8TBps": step_bytes / (ms_step * 1e-3) / 8e12})
        print(f"[entropy30] |S| = {n_s}, K = {K}: S = {r['value']:.5f} +- {r['value_se']:.5f} (Page {page:.5f}), "
              f"{ms_step:.3f} ms per step, {rows[-1]['hbm_GBps_matvec']:.0f} GB/s", file=sys.stderr, flush=True)
    del psi
    torch.cuda.empty_cache()
    return {"workload": "30-qubit Haar state c64, S = first n qubits", "rows": rows}


def run_hbm_sweep(n_steps=10, seed=0, precision="bf16x3",
                  cases=((13, 1, 1), (13, 1, 2), (13, 1, 4), (13, 2, 1), (13, 2, 2), (13, 3, 1),
                         (13, 2, 4), (13, 3, 2), (13, 3, 4), (12, 1, 1), (12, 1, 2), (11, 1, 1), (10, 1, 1)),
                  forms=("lazy", "lazy_two_pass")):
    """(|A|, |B|, K) cases on the 30-qubit state, A = 4.., B right after A;
    each in the one-read form where the shape has it (operator "lazy") and in
    the two-pass form."""
    import torch
    import tnslq_inputs as ti
    dev = torch.device("cuda:0")
    L = 30
    psi = ti.haar_state_torch(L, seed, dev, torch.complex64)
    D = 1 << L
    rows = []
    for na, nb, K in cases:
        a = list(range(4, 4 + na))
        b = list(range(4 + na, 4 + na + nb))
        for form in forms:
            tnslq_logneg(psi, L, a, b, K, 2, precision=precision, seed=seed, want_arrays=False, operator=form)
            r = tnslq_logneg(psi, L, a, b, K, n_steps, precision=precision, seed=seed, want_arrays=False,
                             operator=form)
            d_ab = 1 << (na + nb)
            ms = r["t_matvec_ms"] / r["steps_done"]
            min_bytes = 8 * D + 2 * 8 * d_ab * K
            rows.append({"a_qubits": na, "b_qubits": nb, "probes": K, "operator": form,
                         "path": {0: "split-BF16 MFMA", 1: "two passes", 2: "one read"}[r["streamed"]],
                         "logneg": r["logneg"], "logneg_se": None if K == 1 else r["logneg_se"],
                         "matvec_ms": ms, "min_bytes": min_bytes,
                         "algorithmic_GBps": min_bytes / (ms * 1e-3) / 1e9,
                         "frac_of_8TBps": min_bytes / (ms * 1e-3) / 8e12})
            print(f"[hbm_sweep] |A| = {na}, |B| = {nb}, K = {K}, {form}: {rows[-1]['path']} {ms:.3f} ms per matvec, "
                  f"{rows[-1]['algorithmic_GBps']:.0f} GB/s of minimum bytes, E = {r['logneg']:.4f}",
                  file=sys.stderr, flush=True)
            if not r["streamed"]:
                break
    del psi
    torch.cuda.empty_cache()
    return {"workload": "30-qubit Haar state c64, A = 4.. (|A| qubits), B the next |B| qubits", "precision": precision,
            "steps": n_steps, "rows": rows}


def run_operator_forms(seed=0):
    import torch
    from . import tnslq_logneg as lg
    dev = torch.device("cuda:0")
    cases = [("haar10", 10, [0, 1, 2], [3, 4, 5], 16, 20, False, ["fp64"]),
             ("haar20", 20, list(range(6)), list(range(8, 14)), 32, 40, True, ["fp32", "fp64", "bf16x3"]),
             ("haar24", 24, list(range(7)), list(range(7, 14)), 32, 40, False, ["fp32", "bf16x3"])]
    from tnslq_inputs import haar_state_torch
    rows = []
    for name, L, a, b, K, m, reorth, precs in cases:
        for prec in precs:
            dtype = torch.complex128 if prec == "fp64" else torch.complex64
            psi = haar_state_torch(L, seed, dev, dtype)
            res = {}
            for form in ("lazy", "explicit", "auto"):
                lg(psi, L, a, b, K, 4, reorth=reorth, precision=prec, seed=seed, operator=form, want_arrays=False)
                r = lg(psi, L, a, b, K, m, reorth=reorth, precision=prec, seed=seed, operator=form,
                       want_arrays=False)
                res[form] = r
            row = {"case": name, "n_qubits": L, "d_AB": 1 << (len(a) + len(b)), "d_E": 1 << (L - len(a) - len(b)),
                   "probes": K, "steps": m, "reorth": reorth, "precision": prec,
                   "lazy_s": res["lazy"]["t_total_ms"] / 1e3, "explicit_s": res["explicit"]["t_total_ms"] / 1e3,
                   "explicit_forming_ms": res["explicit"]["t_layout_ms"],
                   "lazy_matvec_ms": res["lazy"]["t_matvec_ms"] / m,
                   "explicit_matvec_ms": res["explicit"]["t_matvec_ms"] / m,
                   "speedup": res["lazy"]["t_total_ms"] / res["explicit"]["t_total_ms"],
                   "auto_explicit": bool(res["auto"]["explicit_operator"]),
                   "E_lazy": res["lazy"]["logneg"], "E_explicit": res["explicit"]["logneg"],
                   "E_difference": res["explicit"]["logneg"] - res["lazy"]["logneg"]}
            rows.append(row)
            print(f"[operator_forms] {name} {prec}: lazy {row['lazy_s']:.4f} s, explicit {row['explicit_s']:.4f} s "
                  f"(forming {row['explicit_forming_ms']:.2f} ms), auto explicit = {row['auto_explicit']}, "
                  f"dE = {row['E_difference']:.2e}", file=sys.stderr, flush=True)
            del psi
            torch.cuda.empty_cache()
    return {"workload": "Haar states, lazy vs explicit rho^{T_B}", "rows": rows}


def run_hbm_peak(reps=10, seed=0):
    import torch
    import tnslq_inputs as ti
    from . import tnslq_spectral_sum
    dev = torch.device("cuda:0")
    out = {}

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        e1.synchronize()
        return e0.elapsed_time(e1) / reps
    n = 1 << 30   # 4 GiB of float32
    src = torch.ones(n, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    ms = timed(lambda: dst.copy_(src))
    out["copy_4GiB"] = {"ms": ms, "GBps": 2 * 4 * n / (ms * 1e-3) / 1e9}
    del dst
    big = torch.ones(2 * n, dtype=torch.float32, device=dev)
    del src
    acc = torch.empty((), dtype=torch.float32, device=dev)
    ms = timed(lambda: torch.sum(big, dim=0, out=acc))
    out["sum_8GiB_float32"] = {"ms": ms, "GBps": 4 * 2 * n / (ms * 1e-3) / 1e9}
    del big, acc
    torch.cuda.empty_cache()
    L = 30
    psi = ti.haar_state_torch(L, seed, dev, torch.complex64)
    for K in (1, 2, 4):
        tnslq_spectral_sum(psi, L, list(range(15)), "purity", K, 2, seed=seed, want_arrays=False)
        r = tnslq_spectral_sum(psi, L, list(range(15)), "purity", K, 20, seed=seed, want_arrays=False)
        ms = r["t_matvec_ms"] / 20
        out[f"entropy_passes_K{K}"] = {"ms_per_step": ms, "GBps": 2 * 8 * (1 << L) / (ms * 1e-3) / 1e9}
    del psi
    torch.cuda.empty_cache()
    for k, v in out.items():
        v["frac_of_8TBps"] = v["GBps"] / 8000.0
        print(f"[hbm_peak] {k}: {v['GBps']:.0f} GB/s ({100 * v['frac_of_8TBps']:.1f}% of 8 TB/s)", file=sys.stderr,
              flush=True)
    return {"workload": "HBM yardstick on one MI355X", "rows": out}


def run_arith_peaks(reps=5, blocks=2048, target_ms=50.0):
    import ctypes
    import os
    import torch
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libtnslq_peak.so")
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with python -m paper_1809_01685_amd.build")
    lib = ctypes.CDLL(path)
    lib.tnslq_peak_flops_per_round.restype = ctypes.c_double
    lib.tnslq_peak_flops_per_round.argtypes = [ctypes.c_int]
    lib.tnslq_peak_launch.restype = ctypes.c_int
    lib.tnslq_peak_launch.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_float, ctypes.c_void_p,
                                      ctypes.c_void_p]
    dev = torch.device("cuda:0")
    out = torch.empty(blocks * 256, dtype=torch.float32, device=dev)
    st = torch.cuda.current_stream(dev)
    # (kind, name, published dense peak in TFLOP/s)
    kinds = [(0, "mfma_bf16_16x16x32", 2500.0), (5, "mfma_bf16_32x32x16", 2500.0), (1, "mfma_f32_16x16x4", 157.3),
             (2, "mfma_f64_16x16x4", 78.6), (3, "valu_fma_f64", 78.6), (4, "valu_fma_f32", 157.3)]
    rows = {}
    for kind, name, peak in kinds:
        per_round = lib.tnslq_peak_flops_per_round(kind) * blocks * 4
        iters = max(1, int(peak * 1e12 * target_ms * 1e-3 / per_round))     # target_ms at the published peak

        def launch():
            rc = lib.tnslq_peak_launch(kind, blocks, iters, ctypes.c_float(1e-3), ctypes.c_void_p(out.data_ptr()),
                                       ctypes.c_void_p(st.cuda_stream))
            if rc != 0:
                raise RuntimeError(f"tnslq_peak_launch({kind}) returned {rc}")
        launch()
        torch.cuda.synchronize()
        rates = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(st)
            launch()
            e1.record(st)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1)
            rates.append(per_round * iters / (ms * 1e-3) / 1e12)
        rates.sort()
        rows[name] = {"iters": iters, "blocks": blocks, "flops_per_launch": per_round * iters,
                      "best_tflops": rates[-1], "median_tflops": rates[len(rates) // 2],
                      "published_tflops": peak, "best_frac_of_published": rates[-1] / peak,
                      "finite": bool(torch.isfinite(out).all().item())}
        print(f"[arith_peaks] {name}: best {rates[-1]:.1f} TFLOP/s, median {rates[len(rates) // 2]:.1f} "
              f"({100 * rates[-1] / peak:.1f}% of the published {peak})", file=sys.stderr, flush=True)
    return {"workload": f"dependent instruction loops, {blocks} workgroups x 4 waves, ~{target_ms} ms each",
            "rows": rows}


def run_mps_blocks(seed=0, n_probes=8, n_steps=40, precision="bf16x3", routes=("dense", "factored"), chis=None):
    """Two blocks of a 100-site random MPS: the dense route (effective state,
    then tnslq_logneg in `precision`) against the factorised operator (FP64),
    both with the fit rule and a 1% target, reorthogonalised (the Krylov
    spaces are small; without it the recurrence drifts before the 40-step
    cap)."""
    import torch
    import tnslq_inputs as ti
    from . import tnslq_logneg, tnslq_logneg_mps, tnslq_mps_effective_state
    dev = torch.device("cuda:0")
    rows = []
    # the last flag: the dense route as well (the gap rows' effective states
    # would need 2^32 amplitudes or more; at chi = 180 it takes 2^31, 32 GiB)
    for chi, a0, la, b0, lb, dense in ((16, 34, 16, 50, 16, True), (32, 34, 16, 50, 16, True),
                                       (16, 32, 16, 52, 16, True), (32, 33, 16, 50, 16, False),
                                       (64, 42, 8, 50, 8, True), (64, 41, 8, 50, 8, False),
                                       (180, 42, 8, 50, 8, True)):
        if chis and chi not in chis:
            continue
        ts = ti.random_mps(100, 2, chi, seed)
        row = {"n_sites": 100, "chi": chi, "A": [a0, a0 + la], "B": [b0, b0 + lb], "gap": b0 - a0 - la}
        if "dense" in routes and dense:
            tnslq_mps_effective_state(ts, a0, la, b0, lb, device=dev)      # warm-up
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            psi, q = tnslq_mps_effective_state(ts, a0, la, b0, lb, device=dev)
            torch.cuda.synchronize()
            t_eff = time.perf_counter() - t0
            qa, qb, qe = q
            t0 = time.perf_counter()
            r = tnslq_logneg(psi, qa + qb + qe, list(range(qa)), list(range(qa, qa + qb)), n_probes, n_steps,
                             precision=precision, seed=seed, stop_tol=0.01, stop_rule="fit", want_arrays=False,
                             reorth=True)
            t_ln = time.perf_counter() - t0
            row.update({"effective_qubits": list(q), "t_effective_state_s": t_eff, "t_logneg_s": t_ln,
                        "logneg": r["logneg"], "logneg_se": r["logneg_se"], "lanczos_err": r["lanczos_err"],
                        "steps": r["steps_done"], "explicit_operator": bool(r["explicit_operator"])})
            print(f"[mps_blocks] chi {chi}, A {row['A']}, B {row['B']}: dense: effective state {q} in "
                  f"{t_eff:.3f} s, E = {r['logneg']:.4f} +- {r['logneg_se']:.4f} after {r['steps_done']} steps "
                  f"in {t_ln:.3f} s", file=sys.stderr, flush=True)
            del psi
            torch.cuda.empty_cache()
        if "factored" in routes:
            tnslq_logneg_mps(ts, a0, la, b0, lb, n_probes, 10, device=dev, seed=seed, want_arrays=False)  # warm-up
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            f = tnslq_logneg_mps(ts, a0, la, b0, lb, n_probes, n_steps, device=dev, seed=seed, stop_tol=0.01,
                                 stop_rule="fit", want_arrays=False, reorth=True)
            t_f = time.perf_counter() - t0
            row["factored"] = {"t_total_s": t_f, "t_layout_ms": f["t_layout_ms"], "t_matvec_ms": f["t_matvec_ms"],
                               "steps": f["steps_done"], "logneg": f["logneg"], "logneg_se": f["logneg_se"],
                               "lanczos_err": f["lanczos_err"], "workspace_bytes": f["workspace_bytes"]}
            print(f"[mps_blocks] chi {chi}, A {row['A']}, B {row['B']}: factored: E = {f['logneg']:.4f} +- "
                  f"{f['logneg_se']:.4f} after {f['steps_done']} steps in {t_f:.3f} s (factors "
                  f"{f['t_layout_ms']:.1f} ms, matvecs {f['t_matvec_ms']:.1f} ms)", file=sys.stderr, flush=True)
            torch.cuda.empty_cache()
            # the same in FP32 (complex64 intermediates, FP32 matrix instructions)
            tnslq_logneg_mps(ts, a0, la, b0, lb, n_probes, 10, device=dev, seed=seed, want_arrays=False,
                             precision="fp32")
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            f = tnslq_logneg_mps(ts, a0, la, b0, lb, n_probes, n_steps, device=dev, seed=seed, stop_tol=0.01,
                                 stop_rule="fit", want_arrays=False, precision="fp32", reorth=True)
            t_f = time.perf_counter() - t0
            row["factored_fp32"] = {"t_total_s": t_f, "t_layout_ms": f["t_layout_ms"],
                                    "t_matvec_ms": f["t_matvec_ms"], "steps": f["steps_done"],
                                    "logneg": f["logneg"], "logneg_se": f["logneg_se"]}
            print(f"[mps_blocks] chi {chi}, A {row['A']}, B {row['B']}: factored FP32: E = {f['logneg']:.4f} +- "
                  f"{f['logneg_se']:.4f} after {f['steps_done']} steps in {t_f:.3f} s (matvecs "
                  f"{f['t_matvec_ms']:.1f} ms)", file=sys.stderr, flush=True)
            torch.cuda.empty_cache()
        rows.append(row)
    return {"workload": "100-site random open-boundary MPS (qubits), two blocks of 8 or 16 sites",
            "precision_dense": precision, "precision_factored": "fp64", "reorth": True, "rows": rows}


def run_mps_long(seed=0, n_probes=2, n_steps=10, chis=(32, 64, 116), lengths=(20, 100, 400), n_sites=1000,
                 rings=True):
    """Long blocks (Sec. VI at the size of its Heisenberg-chain study: 1000
    sites, bonds up to 116, adjacent blocks): seeded random tensors stand in
    for the DMRG ground state.  A = [L/2 - l, L/2), B = [L/2, L/2 + l); the
    blocks' Gram matrices come from transfer sweeps (their explicit sections
    would hold 2^l bond^2 entries).  The factorised operator in FP32, the
    fit rule with a 1% target; t_layout_ms is the whole factor construction
    (environment sweeps, block sweeps, Cholesky factors, normalisation).
    Then rings of 200 sites (bond 8 and 12) with a gap and a 100-site outer
    section."""
    import torch
    import tnslq_inputs as ti
    from . import tnslq_logneg_mps
    dev = torch.device("cuda:0")
    rows = []

    def one(ts, a0, la, b0, lb, row, prec, matvec="auto"):
        t0 = time.perf_counter()
        f = tnslq_logneg_mps(ts, a0, la, b0, lb, n_probes, n_steps, device=dev, seed=seed, stop_tol=0.01,
                             stop_rule="fit", want_arrays=False, precision=prec, matvec=matvec)
        torch.cuda.synchronize()
        row.update({"precision": prec, "matvec": {1: "factors", 2: "network"}[f["mps_matvec"]],
                    "t_total_s": time.perf_counter() - t0, "t_layout_ms": f["t_layout_ms"],
                    "t_matvec_ms": f["t_matvec_ms"], "steps": f["steps_done"],
                    "ms_per_matvec": f["t_matvec_ms"] / max(f["steps_done"], 1), "logneg": f["logneg"],
                    "logneg_se": f["logneg_se"], "lanczos_err": f["lanczos_err"],
                    "workspace_bytes": f["workspace_bytes"]})
        print(f"[mps_long] {row}", file=sys.stderr, flush=True)
        rows.append(row)
        torch.cuda.empty_cache()

    for chi in chis:
        ts = ti.random_mps(n_sites, 2, chi, seed)
        tnslq_logneg_mps(ts, n_sites // 2 - 20, 20, n_sites // 2, 20, n_probes, 2, device=dev, seed=seed,
                         want_arrays=False, precision="fp32")   # warm-up
        for la in lengths:
            c = n_sites // 2
            one(ts, c - la, la, c, la, {"chain": "open", "n_sites": n_sites, "chi": chi, "A": [c - la, c],
                                       "B": [c, c + la]}, "fp32")
    if rings:
        # blocks 40 sites apart on the open chain: the factors' u' = (u, w)
        # is chi^3 wide, the network form keeps E_W (chi^4) apart
        for chi, forms in ((16, ("factors", "network")), (64, ("network",))):
            ts = ti.random_mps(n_sites, 2, chi, seed)
            c = n_sites // 2
            for mv in forms:
                one(ts, c - 100, 80, c + 20, 80, {"chain": "open", "n_sites": n_sites, "chi": chi,
                                                  "A": [c - 100, c - 20], "B": [c + 20, c + 100]}, "fp64", mv)
        for chi in (8, 12, 16, 32):
            ts = ti.random_mps_periodic(200, 2, chi, seed + chi)
            forms = ("factors", "network") if chi == 8 else ("network",)
            for mv in forms:
                one(ts, 10, 40, 60, 40, {"chain": "ring", "n_sites": 200, "chi": chi, "A": [10, 50],
                                         "B": [60, 100], "outer_sites": 110}, "fp64", mv)
    return {"workload": f"seeded random MPS of qubits: open chain of {n_sites} sites, adjacent blocks of "
                        f"{list(lengths)} sites at its centre and 80-site blocks 40 sites apart; rings of 200 "
                        f"sites",
            "n_probes": n_probes, "n_steps": n_steps, "rows": rows}


def _parse_range(s):
    if "-" in s:
        lo, hi = s.split("-")
        return list(range(int(lo), int(hi) + 1))
    return [int(x) for x in s.split(",")]


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    sc = sub.add_parser("scrambling")
    sc.add_argument("--depths", default="1-12")
    sc.add_argument("--precision", default="bf16x3")
    ho = sub.add_parser("heldout26")
    ho.add_argument("--models", default="", help="comma list of checkpoint directories (default: the committed one)")
    hs = sub.add_parser("hbm_sweep")
    hs.add_argument("--cases", default="", help="comma list of |A|:|B|:K (default: the whole sweep)")
    hs.add_argument("--forms", default="lazy,lazy_two_pass")
    hs.add_argument("--steps", type=int, default=10)
    sub.add_parser("operator_forms")
    sl = sub.add_parser("surrogate_latency")
    sl.add_argument("--model", default="")
    sub.add_parser("hbm_peak")
    sp = sub.add_parser("arith_peaks")
    sp.add_argument("--blocks", type=int, default=2048)
    sp.add_argument("--ms", type=float, default=50.0)
    sp = sub.add_parser("mps_blocks")
    sp.add_argument("--routes", default="dense,factored")
    sp.add_argument("--chi", default="", help="comma list: only the rows of these bond dimensions")
    ml = sub.add_parser("mps_long")
    ml.add_argument("--chi", default="32,64,116")
    ml.add_argument("--lengths", default="20,100,400")
    ro = sub.add_parser("rounding")
    ro.add_argument("--depth", type=int, default=8)
    en = sub.add_parser("entropy30")
    en.add_argument("--steps", type=int, default=20)
    args = ap.parse_args(argv)
    if args.cmd == "scrambling":
        out = run_scrambling(_parse_range(args.depths), precision=args.precision)
    elif args.cmd == "mps_blocks":
        out = run_mps_blocks(routes=tuple(args.routes.split(",")),
                             chis=[int(x) for x in args.chi.split(",") if x] or None)
    elif args.cmd == "mps_long":
        out = run_mps_long(chis=[int(x) for x in args.chi.split(",")],
                           lengths=[int(x) for x in args.lengths.split(",")])
    elif args.cmd == "hbm_peak":
        out = run_hbm_peak()
    elif args.cmd == "arith_peaks":
        out = run_arith_peaks(blocks=args.blocks, target_ms=args.ms)
    elif args.cmd == "surrogate_latency":
        out = run_surrogate_latency(model_dir=args.model or None)
    elif args.cmd == "operator_forms":
        out = run_operator_forms()
    elif args.cmd == "hbm_sweep":
        kw = {"forms": tuple(f for f in args.forms.split(",") if f)}
        if args.cases:
            kw["cases"] = tuple(tuple(int(x) for x in c.split(":")) for c in args.cases.split(","))
        out = run_hbm_sweep(n_steps=args.steps, **kw)
    elif args.cmd == "entropy30":
        out = run_entropy30(n_steps=args.steps)
    elif args.cmd == "rounding":
        out = run_rounding(depth=args.depth)
    else:
        out = run_heldout26(models=[m for m in args.models.split(",") if m] or None)
    print(json.dumps(out))


if __name__ == "__main__":
    main(sys.argv[1:])
