"""CPU checks of the C ABI: the library loads, exports every declared entry
point, and validates arguments without touching a device."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1809_01685_amd as T

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "tnslq.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tnslq_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(T.LIB_PATH):
        pytest.skip("libtnslq.so not built")
    return T.lib()


def test_every_declared_symbol_is_exported(L):
    names = _declared()
    assert len(names) >= 15
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(T._SIGS), "binding and header disagree"


def test_version_and_status_strings(L):
    assert T.tnslq_version() == 4
    assert T.tnslq_status_str(0) == "ok"
    assert T.tnslq_status_str(-2) == "invalid partition"
    assert T.tnslq_status_str(-4) == "workspace too small"


def test_workspace_query_and_plan(L):
    o = T.make_options(32, 40, reorth=True, precision="fp32")
    n = T.tnslq_workspace_bytes(T.TNSLQ_C64, 20, list(range(6)), list(range(8, 14)), o)
    # at least the two regrouped copies of psi (2 planes x 4 bytes x 2^20 each)
    assert n >= 2 * 2 * 4 * (1 << 20)
    # the Lanczos basis with reorthogonalisation: 41 slots x 32 probes x 4096 x 16 bytes
    assert n >= 41 * 32 * 4096 * 16
    o2 = T.make_options(32, 40, reorth=False, precision="fp32")
    assert T.tnslq_workspace_bytes(T.TNSLQ_C64, 20, list(range(6)), list(range(8, 14)), o2) < n


def test_operator_form_choice_and_limits(L):
    a20, b20 = list(range(6)), list(range(8, 14))
    ws = {}
    for form in ("auto", "lazy", "explicit"):
        o = T.make_options(32, 40, reorth=True, precision="fp32", operator=form)
        ws[form] = T.tnslq_workspace_bytes(T.TNSLQ_C64, 20, a20, b20, o)
    # the explicit form holds rho^{T_B} (4096^2 complex, FP32 planes) and its
    # dense FP32 precursor
    assert ws["explicit"] >= 2 * 4096 * 4096 * 8
    # at the 20-qubit workload (d_A = d_B = 64, d_E = 256, K = 32, 40 steps)
    # the explicit form does ~3x fewer padded multiply-adds: auto takes it
    assert ws["auto"] == ws["explicit"] != ws["lazy"]
    # d_A d_B = 2^26: only the lazy form
    o = T.make_options(8, 10, precision="bf16x3")
    a30, b30 = list(range(4, 17)), list(range(17, 30))
    assert T.tnslq_workspace_bytes(T.TNSLQ_C64, 30, a30, b30, o) == T.tnslq_workspace_bytes(
        T.TNSLQ_C64, 30, a30, b30, T.make_options(8, 10, precision="bf16x3", operator="lazy"))
    with pytest.raises(T.TnslqError, match="explicit operator"):
        T.tnslq_workspace_bytes(T.TNSLQ_C64, 30, a30, b30, T.make_options(8, 10, precision="bf16x3",
                                                                         operator="explicit"))
    # K d_B <= 8 (streaming regime): auto stays lazy
    o1 = T.make_options(1, 10, operator="auto")
    assert T.tnslq_workspace_bytes(T.TNSLQ_C64, 16, list(range(8)), [8, 9], o1) == T.tnslq_workspace_bytes(
        T.TNSLQ_C64, 16, list(range(8)), [8, 9], T.make_options(1, 10, operator="lazy"))
    p = T._partition(6, [0], [1])
    n = ctypes.c_size_t(0)
    assert L.tnslq_workspace_bytes(0, ctypes.byref(p), ctypes.byref(T.make_options(4, 4, operator=5)),
                                   ctypes.byref(n)) == -1


def test_chunk_cap_sets_the_intermediary_size(L):
    # the intermediary of the lazy form holds d_B x d_E d_B values per probe
    # of a chunk: the workspace shrinks with the cap, by whole chunks
    a30, b30 = list(range(4, 17)), list(range(17, 30))
    ws = {c: T.tnslq_workspace_bytes(T.TNSLQ_C64, 30, a30, b30,
                                     T.make_options(8, 10, precision="bf16x3", chunk_probes=c)) for c in (0, 1, 2, 8)}
    ups = 8192 * 16 * 8192 * 12         # one probe's intermediary, split BF16 (12 B per complex value:
    #                                     re, im and re + im, hi and lo pieces each)
    ypart = 8192 * 8192 * 8             # and its FP32 partial result
    assert ws[0] == ws[2]               # the budget of 2^31 values holds two probes
    assert ws[2] - ws[1] == ups + ypart and ws[8] == ws[0]
    # d_B = 64 < 128: a cap of 3 probes is rounded up to 4 (chunks start on
    # 128-row blocks), so caps 3 and 4 plan alike and 1 becomes 2
    a16, b16 = list(range(0, 8)), list(range(10, 16))
    f = lambda c: T.tnslq_ptmatvec_workspace_bytes(T.TNSLQ_C64, 16, a16, b16, 10, "fp32", c)  # noqa: E731
    assert f(3) == f(4) < f(5) <= f(0) and f(1) == f(2) < f(3)
    with pytest.raises(T.TnslqError) as ei:
        f(-1)
    assert ei.value.status == -1


def test_static_scratch_entry_rejects_what_does_not_fit_before_device_work(L):
    # the 30-qubit problem needs far more than the fixed scratch: a workspace
    # error naming both sizes, with no device touched (none exists here)
    a30, b30 = list(range(4, 17)), list(range(17, 30))
    p = T._partition(30, a30, b30)
    dummy = ctypes.c_void_p(256)
    rc = L.tnslq_ptmatvec_static(dummy, 0, ctypes.byref(p), 8, dummy, ctypes.c_void_p(512), 2, 0, None)
    assert rc == -4
    assert "static scratch holds 67108864" in T.tnslq_last_error()
    # argument errors come first
    assert L.tnslq_ptmatvec_static(dummy, 0, ctypes.byref(p), 8, dummy, dummy, 2, 0, None) == -1
    assert L.tnslq_ptmatvec_static(dummy, 0, ctypes.byref(p), 8, dummy, ctypes.c_void_p(512), 2, -1, None) == -1
    assert T.STATIC_SCRATCH_BYTES == 64 << 20


def test_rho_pt_validates_without_device(L):
    assert T.tnslq_rho_pt_workspace_bytes(T.TNSLQ_C128, 10, [0, 1, 2], [5, 6, 7]) >= 64 * 64 * 16
    with pytest.raises(T.TnslqError) as ei:
        T.tnslq_rho_pt_workspace_bytes(T.TNSLQ_C64, 20, list(range(8)), list(range(8, 15)))
    assert ei.value.status == -1
    with pytest.raises(T.TnslqError) as ei:
        T.tnslq_rho_pt_workspace_bytes(T.TNSLQ_C64, 8, [0, 1], [])
    assert ei.value.status == -2
    p = T._partition(8, [0, 1], [2, 3])
    assert L.tnslq_rho_pt(None, 0, ctypes.byref(p), None, None, 0, None) == -1


@pytest.mark.parametrize("a,b,code", [
    ([0, 1], [1, 2], -2),      # overlap
    ([0, 0], [2], -2),         # repeat
    ([0, 10], [2], -2),        # out of range
])
def test_bad_partitions_rejected(L, a, b, code):
    o = T.make_options(4, 4)
    with pytest.raises(T.TnslqError) as ei:
        T.tnslq_workspace_bytes(T.TNSLQ_C64, 6, a, b, o)
    assert ei.value.status == code


def test_bad_options_rejected(L):
    p = T._partition(6, [0], [1])
    n = ctypes.c_size_t(0)
    for o in (T.make_options(0, 4), T.make_options(4, 0), T.make_options(4, 500), T.make_options(4, 4, precision=9),
              T.make_options(4, 4, stop_rule=7), T.make_options(4, 5, stop_rule="fit"),
              T.make_options(4, 8, stop_tol=0.01, max_probes=-1),
              T.make_options(4, 8, stop_tol=0.01, stop_rule="diff", max_probes=16),
              T.make_options(4, 8, stop_tol=0.0, stop_rule="fit", max_probes=16),
              T.make_options(4, 4, chunk_probes=-1)):
        rc = L.tnslq_workspace_bytes(0, ctypes.byref(p), ctypes.byref(o), ctypes.byref(n))
        assert rc == -1
    assert L.tnslq_workspace_bytes(7, ctypes.byref(p), ctypes.byref(T.make_options(4, 4)), ctypes.byref(n)) == -3


def test_logneg_validates_before_device_work(L):
    p = T._partition(6, [0], [1])
    o = T.make_options(4, 4)
    res = T.Result()
    # NULL psi with a non-trivial partition: argument error, no launch
    rc = L.tnslq_logneg(None, 0, ctypes.byref(p), ctypes.byref(o), None, 0, None, ctypes.byref(res),
                        None, None, None, None, None)
    assert rc == -1
    assert "NULL" in T.tnslq_last_error()


def test_status_codes_and_small_workspace_without_device(L):
    assert [T.tnslq_status_str(c) for c in (-6, -7)] == ["non-finite value", "state not normalised"]
    # a workspace smaller than the plan is refused before psi or the
    # workspace is touched (the pointers here are not device memory)
    p = T._partition(6, [0], [1, 2])
    o = T.make_options(4, 4)
    res = T.Result()
    fake = ctypes.c_void_p(1 << 20)
    rc = L.tnslq_logneg(fake, 0, ctypes.byref(p), ctypes.byref(o), fake, 256, None, ctypes.byref(res),
                        None, None, None, None, None)
    assert rc == T.TNSLQ_E_WORKSPACE and "workspace 256 bytes" in T.tnslq_last_error()
    rc = L.tnslq_ptmatvec(fake, 0, ctypes.byref(p), 2, fake, ctypes.c_void_p(1 << 21), 1, 0, fake, 256, None)
    assert rc == T.TNSLQ_E_WORKSPACE


def test_empty_subsystem_is_exactly_zero_without_device(L):
    p = T._partition(6, [0, 1], [])
    o = T.make_options(3, 5)
    res = T.Result()
    G = np.full(3, -1.0)
    rc = L.tnslq_logneg(None, 0, ctypes.byref(p), ctypes.byref(o), None, 0, None, ctypes.byref(res),
                        G.ctypes.data_as(ctypes.c_void_p), None, None, None, None)
    assert rc == 0
    assert res.logneg == 0.0 and res.trace_norm == 1.0
    assert np.all(G == 1.0)


def test_mlp_argument_checks(L):
    n = ctypes.c_size_t(0)
    assert L.tnslq_mlp_workspace_bytes(0, ctypes.byref(n)) == -1
    assert L.tnslq_mlp_workspace_bytes(64, ctypes.byref(n)) == 0 and n.value > 64 * 256 * 4
    assert L.tnslq_mlp_adam(None, None, None, None, 1, 1e-3, None) == -1


def test_binding_structs_match_the_header(tmp_path):
    # the ctypes mirrors must have the C layout: compile a probe of the header
    # with the host compiler and compare sizes and field offsets
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    structs = {"tnslq_partition": T.Partition, "tnslq_options": T.Options, "tnslq_result": T.Result,
               "tnslq_spectral_result": T.SpectralResult, "tnslq_partition_dims": T.PartitionDims,
               "tnslq_mps": T.Mps}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "tnslq.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} sizeof %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "probe.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "probe"
    subprocess.run([cc, "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cname, py in structs.items():
        assert got[(cname, "sizeof")] == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)


def test_spectral_sum_validates_and_handles_trivial_subsystems_without_device(L):
    import ctypes as C
    o = T.make_options(3, 5, precision="fp64")
    res = T.SpectralResult()
    G = np.full(3, -1.0)
    for fn, want in ((T.TNSLQ_F_ENTROPY, 0.0), (T.TNSLQ_F_PURITY, 1.0)):
        for s in ([], [0, 1, 2, 3]):
            arr = (C.c_int * 4)(*s) if s else None
            rc = L.tnslq_spectral_sum(None, 0, 4, C.cast(arr, C.c_void_p) if arr else None, len(s), fn,
                                      C.byref(o), None, 0, None, C.byref(res), G.ctypes.data_as(C.c_void_p),
                                      None, None, None, None)
            assert rc == 0 and res.value == want and np.all(G == want)
    arr = (C.c_int * 2)(0, 1)
    bad = [(o, 7), (T.make_options(3, 5, precision="fp32"), 1), (T.make_options(3, 5, precision="fp64", stop_tol=0.1), 1)]
    for oo, fn in bad:
        rc = L.tnslq_spectral_sum(None, 0, 4, C.cast(arr, C.c_void_p), 2, fn, C.byref(oo), None, 0, None,
                                  C.byref(res), None, None, None, None, None)
        assert rc == -1, (fn, oo.precision)
    # NULL psi on a real subsystem: argument error before any launch
    rc = L.tnslq_spectral_sum(None, 0, 4, C.cast(arr, C.c_void_p), 2, 1, C.byref(o), None, 0, None,
                              C.byref(res), None, None, None, None, None)
    assert rc == -1 and "NULL" in T.tnslq_last_error()
    rep = (C.c_int * 2)(1, 1)
    n = C.c_size_t(0)
    assert L.tnslq_spectral_workspace_bytes(0, 4, C.cast(rep, C.c_void_p), 2, C.byref(o), C.byref(n)) == -2


def test_spectral_workspace_uses_the_smaller_side(L):
    o = T.make_options(4, 10, precision="fp64")
    small = T.tnslq_spectral_workspace_bytes(T.TNSLQ_C64, 16, [0, 1, 2], o)
    large = T.tnslq_spectral_workspace_bytes(T.TNSLQ_C64, 16, list(range(3, 16)), o)
    assert small == large > 2 * 8 * (1 << 16)


def test_dims_entry_points_validate_without_device(L):
    o = T.make_options(4, 8, precision="fp64")
    # qutrits: 3^4 = 81 amplitudes, d_A d_B = 9
    assert T.tnslq_workspace_bytes_dims(T.TNSLQ_C128, [3, 3, 3, 3], [0], [2], o) > 0
    with pytest.raises(T.TnslqError, match="explicit operator only"):
        T.tnslq_workspace_bytes_dims(T.TNSLQ_C128, [3, 3, 3, 3], [0], [2], T.make_options(4, 8, operator="lazy"))
    for dims, a, b in (([3, 1, 3], [0], [2]), ([3, 3], [0], [0]), ([3, 3], [0], [5])):
        with pytest.raises(T.TnslqError) as ei:
            T.tnslq_workspace_bytes_dims(T.TNSLQ_C128, dims, a, b, o)
        assert ei.value.status == -2
    # d_A d_B = 3^9 > 16384
    with pytest.raises(T.TnslqError, match="exceeds"):
        T.tnslq_workspace_bytes_dims(T.TNSLQ_C64, [3] * 10, list(range(5)), list(range(5, 9)), o)
    assert T.tnslq_workspace_bytes_dims(T.TNSLQ_C64, [3, 3], [0], [], o) == 0


def test_mps_sizes_and_validation_without_device(L):
    import ctypes as C

    def desc(phys, bond):
        pp = (C.c_int * len(phys))(*phys)
        bb = (C.c_int * len(bond))(*bond)
        m = T.Mps(len(phys), pp, bb, None)
        m._keep = (pp, bb)
        return m
    # 12 qubits, bond 4: A = [2, 6) (2^4 = 16 = 4 x 4, not compressed), B = [6, 10)
    phys, bond = [2] * 12, [1, 2, 4, 4, 4, 4, 4, 4, 4, 4, 4, 2, 1]
    q = (C.c_int * 3)()
    n = C.c_size_t(0)
    assert L.tnslq_mps_effective_state_size(C.byref(desc(phys, bond)), 2, 4, 6, 4, q, C.byref(n)) == 0
    assert list(q) == [4, 4, 4] and n.value > 0          # d_E' = bond[2] bond[10] = 16
    # blocks out of order, or past the chain
    for a0, na, b0, nb in ((6, 4, 2, 4), (2, 5, 6, 4), (2, 4, 10, 3)):
        assert L.tnslq_mps_effective_state_size(C.byref(desc(phys, bond)), a0, na, b0, nb, q, C.byref(n)) == -2
    bad = list(bond)
    bad[0] = 2
    assert L.tnslq_mps_effective_state_size(C.byref(desc(phys, bad)), 2, 4, 6, 4, q, C.byref(n)) == -1
    assert L.tnslq_mps_effective_state(C.byref(desc(phys, bond)), 2, 4, 6, 4, None, None, 0, None) == -1


def test_mps_rings_and_section_routes_without_device(L):
    import ctypes as C

    def desc(phys, bond, sections=0):
        pp = (C.c_int * len(phys))(*phys)
        bb = (C.c_int * len(bond))(*bond)
        m = T.Mps(len(phys), pp, bb, None, sections)
        m._keep = (pp, bb)
        return m
    q = (C.c_int * 3)()
    n = C.c_size_t(0)
    # a ring of 10 qubits, every bond 3: A = [1, 4), B = [5, 8), outer
    # section [8, 10) + [0, 1) (2^3 = 8 <= 9: kept whole, d_Z = 8), gap [4, 5)
    # (2 <= 9, d_W = 2); A and B compressed (8 <= 9: no, kept whole)
    phys, bond = [2] * 10, [3] * 11
    assert L.tnslq_mps_effective_state_size(C.byref(desc(phys, bond)), 1, 3, 5, 3, q, C.byref(n)) == 0
    assert list(q) == [3, 3, 4]                      # E' = (w, z) = 2 x 8
    # blocks covering the ring: the outer section is the identity, E' = 1
    assert L.tnslq_mps_effective_state_size(C.byref(desc(phys, bond)), 0, 5, 5, 5, q, C.byref(n)) == 0
    assert list(q) == [4, 4, 0]                      # compressed blocks: 3 x 3 = 9 -> 16
    # route values outside the enumeration
    for bad in (-1, 3):
        assert L.tnslq_mps_effective_state_size(C.byref(desc(phys, bond, bad)), 1, 3, 5, 3, q, C.byref(n)) == -1
    # 200 qubits, bond 4: blocks of 80 sites reach only the transfer route
    phys, bond = [2] * 200, [1, 2] + [4] * 197 + [2, 1]
    assert L.tnslq_mps_effective_state_size(C.byref(desc(phys, bond, 0)), 10, 80, 90, 80, q, C.byref(n)) == 0
    assert list(q) == [4, 4, 4]
    assert L.tnslq_mps_effective_state_size(C.byref(desc(phys, bond, 2)), 10, 80, 90, 80, q, C.byref(n)) == 0
    assert L.tnslq_mps_effective_state_size(C.byref(desc(phys, bond, 1)), 10, 80, 90, 80, q, C.byref(n)) == -1
    assert "transfer route" in T.tnslq_last_error()
    # the matvec form: out-of-range values are argument errors; on a ring
    # with a gap the network form needs far less room than the factors
    ring = [np.zeros((8, 2, 8)) for _ in range(40)]
    o = T.make_options(2, 4, precision="fp64")
    for bad in (-1, 3):
        m = T._mps_desc(ring)
        m.matvec = bad
        assert L.tnslq_workspace_bytes_mps(C.byref(m), 2, 10, 16, 10, C.byref(o), C.byref(n)) == -1
    w_net = T.tnslq_workspace_bytes_mps(ring, 2, 10, 16, 10, o, matvec="network")
    w_pq = T.tnslq_workspace_bytes_mps(ring, 2, 10, 16, 10, o, matvec="factors")
    assert T.tnslq_workspace_bytes_mps(ring, 2, 10, 16, 10, o) == w_net < w_pq / 10
    # blocks whose compressed dimension is not a power of two and whose
    # probes do not fit one chunk (d_A' = d_B' = 13456 at bond 116, 2 probes)
    bond = [1] + [min(2 ** min(i, 60 - i), 116) for i in range(1, 60)] + [1]
    tensors = [np.zeros((bond[i], 2, bond[i + 1])) for i in range(60)]
    assert T.tnslq_workspace_bytes_mps(tensors, 10, 20, 30, 20, T.make_options(2, 4, precision="fp32")) > 0
    # factored matrices up to 16384 wide: bond 128 around a compressed block
    # of 17 sites (2^17 > 128 x 128; with bond 256, 2^17 > 256 x 256 too)
    o = T.make_options(2, 4, precision="fp64")
    for chi, ok in ((128, True), (256, False)):
        bond = [1] + [min(2 ** min(i, 40 - i), chi) for i in range(1, 40)] + [1]
        tensors = [np.zeros((bond[i], 2, bond[i + 1])) for i in range(40)]
        if ok:
            assert T.tnslq_workspace_bytes_mps(tensors, 8, 17, 25, 13, o) > 0
        else:
            with pytest.raises(T.TnslqError, match="16384"):
                T.tnslq_workspace_bytes_mps(tensors, 8, 17, 25, 13, o)


def test_factored_mps_workspace_and_validation_without_device(L):
    import ctypes as C
    # the same chain: the factorised route needs no room for the dense state
    phys, bond = [2] * 12, [1, 2, 4, 4, 4, 4, 4, 4, 4, 4, 4, 2, 1]
    tensors = [np.zeros((bond[i], 2, bond[i + 1])) for i in range(12)]
    o = T.make_options(8, 20, precision="fp64")
    n = T.tnslq_workspace_bytes_mps(tensors, 2, 4, 6, 4, o)
    # Lanczos vectors of d_A' d_B' = 256 entries: three slots of 8 probes at least
    assert n >= 3 * 8 * 256 * 16
    # more probes need more room; reorthogonalisation keeps every vector
    assert T.tnslq_workspace_bytes_mps(tensors, 2, 4, 6, 4, T.make_options(16, 20, precision="fp64")) > n
    assert T.tnslq_workspace_bytes_mps(tensors, 2, 4, 6, 4, T.make_options(8, 20, True, precision="fp64")) > n
    # FP32 halves the intermediates and adds complex64 copies of the factors
    n32 = T.tnslq_workspace_bytes_mps(tensors, 2, 4, 6, 4, T.make_options(8, 20, precision="fp32"))
    assert 0 < n32
    for bad in (T.make_options(8, 20, precision="bf16x3"), T.make_options(8, 20, precision="fp64", operator="lazy")):
        with pytest.raises(T.TnslqError):
            T.tnslq_workspace_bytes_mps(tensors, 2, 4, 6, 4, bad)
    with pytest.raises(T.TnslqError):
        T.tnslq_workspace_bytes_mps(tensors, 6, 4, 2, 4, o)
    desc = T._mps_desc(tensors)
    res = T.Result()
    assert L.tnslq_logneg_mps(C.byref(desc), 2, 4, 6, 4, C.byref(o), None, 0, None, C.byref(res), None, None, None,
                              None, None) == -1         # tensors NULL
    assert L.tnslq_logneg_mps(C.byref(desc), 2, 4, 6, 4, C.byref(o), None, 0, None, None, None, None, None, None,
                              None) == -1               # result NULL
