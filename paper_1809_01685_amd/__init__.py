"""Python binding of libtnslq (TNSLQ logarithmic negativity on MI355X).

Argument marshalling only: every step of the computation runs in the HIP
kernels of ``libtnslq.so`` behind the C ABI declared in ``include/tnslq.h``.
torch supplies device memory and the current stream.  The functions keep the
C names; importing works without a GPU (the library is loaded on first use),
and a missing library raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import math
import os
from typing import Dict, Optional, Sequence

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libtnslq.so")

TNSLQ_OK = 0
TNSLQ_E_ARG, TNSLQ_E_PARTITION, TNSLQ_E_DTYPE, TNSLQ_E_WORKSPACE = -1, -2, -3, -4
TNSLQ_E_DEVICE, TNSLQ_E_NONFINITE, TNSLQ_E_STATE = -5, -6, -7
TNSLQ_C64, TNSLQ_C128 = 0, 1
TNSLQ_FP64, TNSLQ_FP32, TNSLQ_BF16X3, TNSLQ_BF16X6 = 0, 1, 2, 3
PRECISIONS = {"fp64": TNSLQ_FP64, "fp32": TNSLQ_FP32, "bf16x3": TNSLQ_BF16X3, "bf16x6": TNSLQ_BF16X6}
TNSLQ_STOP_DIFF, TNSLQ_STOP_FIT = 0, 1
STOP_RULES = {"diff": TNSLQ_STOP_DIFF, "fit": TNSLQ_STOP_FIT}
TNSLQ_OPERATOR_AUTO, TNSLQ_OPERATOR_LAZY, TNSLQ_OPERATOR_EXPLICIT, TNSLQ_OPERATOR_LAZY_TWO_PASS = 0, 1, 2, 3
OPERATORS = {"auto": TNSLQ_OPERATOR_AUTO, "lazy": TNSLQ_OPERATOR_LAZY, "explicit": TNSLQ_OPERATOR_EXPLICIT,
             "lazy_two_pass": TNSLQ_OPERATOR_LAZY_TWO_PASS}
TNSLQ_FIT_WINDOW, TNSLQ_FIT_MIN_POINTS = 8, 5
TNSLQ_F_ABS, TNSLQ_F_ENTROPY, TNSLQ_F_PURITY = 0, 1, 2
FUNCTIONS = {"entropy": TNSLQ_F_ENTROPY, "purity": TNSLQ_F_PURITY}
MLP_NIN, MLP_NHID, MLP_NOUT, MLP_NPARAMS = 19, 256, 2, 71426


class TnslqError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__(f"{where}: status {status}: {detail}")
        self.status = status


class Partition(ctypes.Structure):
    _fields_ = [("n_qubits", ctypes.c_int), ("a", ctypes.POINTER(ctypes.c_int)), ("n_a", ctypes.c_int),
                ("b", ctypes.POINTER(ctypes.c_int)), ("n_b", ctypes.c_int)]


class PartitionDims(ctypes.Structure):
    _fields_ = [("n_sites", ctypes.c_int), ("dims", ctypes.POINTER(ctypes.c_int)), ("a", ctypes.POINTER(ctypes.c_int)),
                ("n_a", ctypes.c_int), ("b", ctypes.POINTER(ctypes.c_int)), ("n_b", ctypes.c_int)]


class Mps(ctypes.Structure):
    _fields_ = [("n_sites", ctypes.c_int), ("phys", ctypes.POINTER(ctypes.c_int)), ("bond", ctypes.POINTER(ctypes.c_int)),
                ("tensors", ctypes.c_void_p), ("sections", ctypes.c_int), ("matvec", ctypes.c_int)]


MPS_SECTIONS = {"auto": 0, "explicit": 1, "transfer": 2}
MPS_MATVEC = {"auto": 0, "factors": 1, "network": 2}


class Options(ctypes.Structure):
    _fields_ = [("n_probes", ctypes.c_int), ("n_steps", ctypes.c_int), ("reorth", ctypes.c_int),
                ("precision", ctypes.c_int), ("seed", ctypes.c_uint64), ("probe_offset", ctypes.c_uint64),
                ("stop_tol", ctypes.c_double), ("stop_rule", ctypes.c_int), ("operator_form", ctypes.c_int),
                ("max_probes", ctypes.c_int), ("chunk_probes", ctypes.c_int)]


class SpectralResult(ctypes.Structure):
    _fields_ = [("value", ctypes.c_double), ("value_se", ctypes.c_double), ("steps_done", ctypes.c_int),
                ("steps_min", ctypes.c_int), ("complement", ctypes.c_int), ("n_qubits_side", ctypes.c_int),
                ("t_layout_ms", ctypes.c_double), ("t_matvec_ms", ctypes.c_double),
                ("t_lanczos_ms", ctypes.c_double), ("t_total_ms", ctypes.c_double)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class Result(ctypes.Structure):
    _fields_ = [("logneg", ctypes.c_double), ("logneg_se", ctypes.c_double), ("trace_norm", ctypes.c_double),
                ("trace_norm_se", ctypes.c_double), ("steps_done", ctypes.c_int), ("steps_min", ctypes.c_int),
                ("swapped_ab", ctypes.c_int), ("n_matvecs", ctypes.c_int), ("n_contract_launches", ctypes.c_int),
                ("t_layout_ms", ctypes.c_double), ("t_matvec_ms", ctypes.c_double),
                ("t_contract1_ms", ctypes.c_double), ("t_contract2_ms", ctypes.c_double),
                ("t_lanczos_ms", ctypes.c_double), ("t_total_ms", ctypes.c_double),
                ("lanczos_err", ctypes.c_double), ("streamed", ctypes.c_int), ("explicit_operator", ctypes.c_int),
                ("n_probes_used", ctypes.c_int), ("mps_matvec", ctypes.c_int)]

    def as_dict(self) -> Dict[str, float]:
        return {name: getattr(self, name) for name, _ in self._fields_}


_lib = None
_VP, _SZ, _I, _D, _F, _U64, _I64 = (ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int, ctypes.c_double,
                                    ctypes.c_float, ctypes.c_uint64, ctypes.c_int64)
_SIGS = {
    "tnslq_status_str": (ctypes.c_char_p, [_I]),
    "tnslq_last_error": (ctypes.c_char_p, []),
    "tnslq_version": (_I, []),
    "tnslq_workspace_bytes": (_I, [_I, ctypes.POINTER(Partition), ctypes.POINTER(Options), ctypes.POINTER(_SZ)]),
    "tnslq_logneg": (_I, [_VP, _I, ctypes.POINTER(Partition), ctypes.POINTER(Options), _VP, _SZ, _VP,
                          ctypes.POINTER(Result), _VP, _VP, _VP, _VP, _VP]),
    "tnslq_ptmatvec_workspace_bytes": (_I, [_I, ctypes.POINTER(Partition), _I, _I, _I, ctypes.POINTER(_SZ)]),
    "tnslq_ptmatvec": (_I, [_VP, _I, ctypes.POINTER(Partition), _I, _VP, _VP, _I, _I, _VP, _SZ, _VP]),
    "tnslq_ptmatvec_static": (_I, [_VP, _I, ctypes.POINTER(Partition), _I, _VP, _VP, _I, _I, _VP]),
    "tnslq_workspace_bytes_dims": (_I, [_I, ctypes.POINTER(PartitionDims), ctypes.POINTER(Options),
                                        ctypes.POINTER(_SZ)]),
    "tnslq_logneg_dims": (_I, [_VP, _I, ctypes.POINTER(PartitionDims), ctypes.POINTER(Options), _VP, _SZ, _VP,
                               ctypes.POINTER(Result), _VP, _VP, _VP, _VP, _VP]),
    "tnslq_rho_pt_dims_workspace_bytes": (_I, [_I, ctypes.POINTER(PartitionDims), ctypes.POINTER(_SZ)]),
    "tnslq_rho_pt_dims": (_I, [_VP, _I, ctypes.POINTER(PartitionDims), _VP, _VP, _SZ, _VP]),
    "tnslq_mps_effective_state_size": (_I, [ctypes.POINTER(Mps), _I, _I, _I, _I, ctypes.POINTER(_I),
                                            ctypes.POINTER(_SZ)]),
    "tnslq_mps_effective_state": (_I, [ctypes.POINTER(Mps), _I, _I, _I, _I, _VP, _VP, _SZ, _VP]),
    "tnslq_workspace_bytes_mps": (_I, [ctypes.POINTER(Mps), _I, _I, _I, _I, ctypes.POINTER(Options),
                                       ctypes.POINTER(_SZ)]),
    "tnslq_logneg_mps": (_I, [ctypes.POINTER(Mps), _I, _I, _I, _I, ctypes.POINTER(Options), _VP, _SZ, _VP,
                              ctypes.POINTER(Result), _VP, _VP, _VP, _VP, _VP]),
    "tnslq_rho_pt_workspace_bytes": (_I, [_I, ctypes.POINTER(Partition), ctypes.POINTER(_SZ)]),
    "tnslq_rho_pt": (_I, [_VP, _I, ctypes.POINTER(Partition), _VP, _VP, _SZ, _VP]),
    "tnslq_quadrature": (_I, [_VP, _VP, _VP, _I, _I, _VP, _VP]),
    "tnslq_probes": (_I, [_U64, _U64, _I, _I64, _VP, _VP]),
    "tnslq_mlp_workspace_bytes": (_I, [_I, ctypes.POINTER(_SZ)]),
    "tnslq_mlp_forward": (_I, [_VP, _VP, _VP, _I, _VP, _VP, _SZ, _VP]),
    "tnslq_mlp_loss_grad": (_I, [_VP, _VP, _VP, _VP, _I, _VP, _VP, _VP, _SZ, _VP]),
    "tnslq_mlp_adam": (_I, [_VP, _VP, _VP, _VP, _I, _F, _VP]),
    "tnslq_mlp_train": (_I, [_VP, _VP, _VP, _VP, _VP, _VP, _VP, _I, _I, _I, _F, _VP, _VP, _SZ, _VP]),
    "tnslq_logneg_surrogate": (_I, [_VP, _I, ctypes.POINTER(Partition), ctypes.POINTER(Options), _VP, _VP, _F, _I,
                                    _D, _VP, _SZ, _VP, ctypes.POINTER(Result), _VP]),
    "tnslq_spectral_workspace_bytes": (_I, [_I, _I, _VP, _I, ctypes.POINTER(Options), ctypes.POINTER(_SZ)]),
    "tnslq_spectral_sum": (_I, [_VP, _I, _I, _VP, _I, _I, ctypes.POINTER(Options), _VP, _SZ, _VP,
                                ctypes.POINTER(SpectralResult), _VP, _VP, _VP, _VP, _VP]),
    "tnslq_mutual_information_workspace_bytes": (_I, [_I, ctypes.POINTER(Partition), ctypes.POINTER(Options),
                                                      ctypes.POINTER(_SZ)]),
    "tnslq_mutual_information": (_I, [_VP, _I, ctypes.POINTER(Partition), ctypes.POINTER(Options), _VP, _SZ, _VP,
                                      _VP]),
}


def lib():
    """Load libtnslq.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1809_01685_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(rc: int, where: str):
    if rc != TNSLQ_OK:
        detail = lib().tnslq_last_error().decode()
        raise TnslqError(rc, where, detail or lib().tnslq_status_str(rc).decode())


def _partition_dims(dims: Sequence[int], a: Sequence[int], b: Sequence[int]):
    dd = (ctypes.c_int * max(1, len(dims)))(*dims)
    aa = (ctypes.c_int * max(1, len(a)))(*a)
    bb = (ctypes.c_int * max(1, len(b)))(*b)
    p = PartitionDims(len(dims), dd, aa, len(a), bb, len(b))
    p._keep = (dd, aa, bb)
    return p


def _partition(n_qubits: int, a: Sequence[int], b: Sequence[int]):
    aa = (ctypes.c_int * max(1, len(a)))(*a)
    bb = (ctypes.c_int * max(1, len(b)))(*b)
    p = Partition(n_qubits, aa, len(a), bb, len(b))
    p._keep = (aa, bb)  # keep the arrays alive with the struct
    return p


def _dtype_code(t) -> int:
    import torch
    if t.dtype == torch.complex64:
        return TNSLQ_C64
    if t.dtype == torch.complex128:
        return TNSLQ_C128
    raise TypeError(f"psi must be complex64 or complex128, got {t.dtype}")


def _prec(p) -> int:
    return PRECISIONS[p] if isinstance(p, str) else int(p)


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _workspace(nbytes: int, device, ws=None):
    """The caller's workspace as given (the library checks its size), else a
    new one of nbytes."""
    import torch
    if ws is not None:
        return ws
    return torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)


def _check_device_tensor(t, name):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


# ----------------------------------------------------------------- utilities
def tnslq_version() -> int:
    return lib().tnslq_version()


def tnslq_status_str(status: int) -> str:
    return lib().tnslq_status_str(status).decode()


def tnslq_last_error() -> str:
    return lib().tnslq_last_error().decode()


def _rule(stop_rule) -> int:
    if isinstance(stop_rule, str):
        return STOP_RULES[stop_rule]
    return int(stop_rule)


def _operator(operator) -> int:
    if isinstance(operator, str):
        return OPERATORS[operator]
    return int(operator)


def make_options(n_probes: int, n_steps: int, reorth: bool = False, precision="fp32", seed: int = 0,
                 probe_offset: int = 0, stop_tol: float = 0.0, stop_rule="diff", operator="auto",
                 max_probes: int = 0, chunk_probes: int = 0) -> Options:
    return Options(int(n_probes), int(n_steps), int(bool(reorth)), _prec(precision), int(seed) & (2**64 - 1),
                   int(probe_offset), float(stop_tol), _rule(stop_rule), _operator(operator), int(max_probes),
                   int(chunk_probes))


def tnslq_workspace_bytes(dtype: int, n_qubits: int, a, b, opts: Options) -> int:
    n = ctypes.c_size_t(0)
    p = _partition(n_qubits, a, b)
    _check(lib().tnslq_workspace_bytes(int(dtype), ctypes.byref(p), ctypes.byref(opts), ctypes.byref(n)),
           "tnslq_workspace_bytes")
    return n.value


# ------------------------------------------------------------- logneg
def tnslq_logneg(psi, n_qubits: int, a, b, n_probes: int, n_steps: int, reorth: bool = False, precision="fp32",
                 seed: int = 0, probe_offset: int = 0, stop_tol: float = 0.0, workspace=None, stream=None,
                 want_arrays: bool = True, stop_rule="diff", operator="auto", max_probes: int = 0,
                 chunk_probes: int = 0) -> Dict[str, object]:
    """SLQ estimate of log2 Tr|rho_AB^{T_B}| of the device state ``psi``.

    With ``max_probes`` > ``n_probes`` (fit rule, ``stop_tol`` > 0) blocks of
    ``n_probes`` probes are added until the estimate meets the target; only
    ``G`` (one value per probe used) is returned among the arrays."""
    import numpy as np
    _check_device_tensor(psi, "psi")
    if psi.numel() != 1 << n_qubits:
        raise ValueError("psi has the wrong length")
    dt = _dtype_code(psi)
    opts = make_options(n_probes, n_steps, reorth, precision, seed, probe_offset, stop_tol, stop_rule, operator,
                        max_probes, chunk_probes)
    if max_probes > n_probes:
        p = _partition(n_qubits, a, b)
        ws = _workspace(tnslq_workspace_bytes(dt, n_qubits, a, b, opts), psi.device, workspace)
        res = Result()
        G = np.zeros(max_probes)
        rc = lib().tnslq_logneg(_ptr(psi), dt, ctypes.byref(p), ctypes.byref(opts), _ptr(ws), ws.numel(),
                                _stream(stream), ctypes.byref(res), G.ctypes.data_as(ctypes.c_void_p), None, None,
                                None, None)
        _check(rc, "tnslq_logneg")
        out: Dict[str, object] = res.as_dict()
        out["G"] = G[:res.n_probes_used].copy()
        out["workspace_bytes"] = ws.numel()
        return out
    p = _partition(n_qubits, a, b)
    need = tnslq_workspace_bytes(dt, n_qubits, a, b, opts)
    ws = _workspace(need, psi.device, workspace)
    res = Result()
    K, m = n_probes, n_steps
    G = np.zeros(K)
    al = np.zeros((K, m))
    be = np.zeros((K, m + 1))
    F = np.zeros((K, m))
    st = np.zeros(K, dtype=np.int32)
    host = (lambda x: x.ctypes.data_as(ctypes.c_void_p)) if want_arrays else (lambda x: ctypes.c_void_p(0))
    rc = lib().tnslq_logneg(_ptr(psi), dt, ctypes.byref(p), ctypes.byref(opts), _ptr(ws), ws.numel(),
                            _stream(stream), ctypes.byref(res), host(G), host(al), host(be), host(F), host(st))
    _check(rc, "tnslq_logneg")
    out: Dict[str, object] = res.as_dict()
    if want_arrays:
        out.update({"G": G, "alpha": al, "beta": be, "F": F, "steps": st})
    out["workspace_bytes"] = need
    return out


# ------------------------------------------------------------- matvec
def tnslq_ptmatvec_workspace_bytes(dtype: int, n_qubits: int, a, b, n_vectors: int, precision="fp32",
                                   chunk_vectors: int = 0) -> int:
    n = ctypes.c_size_t(0)
    p = _partition(n_qubits, a, b)
    _check(lib().tnslq_ptmatvec_workspace_bytes(int(dtype), ctypes.byref(p), int(n_vectors), _prec(precision),
                                                int(chunk_vectors), ctypes.byref(n)), "tnslq_ptmatvec_workspace_bytes")
    return n.value


def tnslq_ptmatvec(psi, n_qubits: int, a, b, X, precision="fp32", workspace=None, stream=None, Y=None,
                   chunk_vectors: int = 0):
    """Y = rho_AB^{T_B} X for device complex128 X of shape (K, d_A d_B)."""
    import torch
    _check_device_tensor(psi, "psi")
    _check_device_tensor(X, "X")
    if X.dtype != torch.complex128 or X.dim() != 2:
        raise TypeError("X must be a 2-D complex128 device tensor")
    dt = _dtype_code(psi)
    K = X.shape[0]
    need = tnslq_ptmatvec_workspace_bytes(dt, n_qubits, a, b, K, precision, chunk_vectors)
    ws = _workspace(need, psi.device, workspace)
    if Y is None:
        Y = torch.empty_like(X)
    p = _partition(n_qubits, a, b)
    _check(lib().tnslq_ptmatvec(_ptr(psi), dt, ctypes.byref(p), K, _ptr(X), _ptr(Y), _prec(precision),
                                int(chunk_vectors), _ptr(ws), ws.numel(), _stream(stream)), "tnslq_ptmatvec")
    return Y


STATIC_SCRATCH_BYTES = 64 << 20


def tnslq_ptmatvec_static(psi, n_qubits: int, a, b, X, precision="fp32", stream=None, Y=None, chunk_vectors: int = 0):
    """tnslq_ptmatvec on the library's fixed per-GPU scratch (no workspace,
    nothing allocated by the library; ``Y`` is allocated here when not given)."""
    import torch
    _check_device_tensor(psi, "psi")
    _check_device_tensor(X, "X")
    if X.dtype != torch.complex128 or X.dim() != 2:
        raise TypeError("X must be a 2-D complex128 device tensor")
    if Y is None:
        Y = torch.empty_like(X)
    p = _partition(n_qubits, a, b)
    _check(lib().tnslq_ptmatvec_static(_ptr(psi), _dtype_code(psi), ctypes.byref(p), X.shape[0], _ptr(X), _ptr(Y),
                                       _prec(precision), int(chunk_vectors), _stream(stream)),
           "tnslq_ptmatvec_static")
    return Y


# ------------------------------------------------- sites of any dimension
def tnslq_workspace_bytes_dims(dtype: int, dims, a, b, opts: Options) -> int:
    n = ctypes.c_size_t(0)
    p = _partition_dims(dims, a, b)
    _check(lib().tnslq_workspace_bytes_dims(int(dtype), ctypes.byref(p), ctypes.byref(opts), ctypes.byref(n)),
           "tnslq_workspace_bytes_dims")
    return n.value


def tnslq_logneg_dims(psi, dims, a, b, n_probes: int, n_steps: int, reorth: bool = False, precision="fp32",
                      seed: int = 0, probe_offset: int = 0, stop_tol: float = 0.0, workspace=None, stream=None,
                      stop_rule="diff", operator="auto", max_probes: int = 0) -> Dict[str, object]:
    """tnslq_logneg for a state on sites with dims[s] levels (explicit operator)."""
    import numpy as np
    _check_device_tensor(psi, "psi")
    if psi.numel() != int(np.prod(list(dims), dtype=np.int64)):
        raise ValueError("psi has the wrong length")
    dt = _dtype_code(psi)
    opts = make_options(n_probes, n_steps, reorth, precision, seed, probe_offset, stop_tol, stop_rule, operator,
                        max_probes)
    p = _partition_dims(dims, a, b)
    ws = _workspace(tnslq_workspace_bytes_dims(dt, dims, a, b, opts), psi.device, workspace)
    res = Result()
    K, m = n_probes, n_steps
    loop = max_probes > n_probes
    G = np.zeros(max(K, max_probes))
    al, be, F = np.zeros((K, m)), np.zeros((K, m + 1)), np.zeros((K, m))
    st = np.zeros(K, dtype=np.int32)
    host = (lambda x: ctypes.c_void_p(0)) if loop else (lambda x: x.ctypes.data_as(ctypes.c_void_p))
    rc = lib().tnslq_logneg_dims(_ptr(psi), dt, ctypes.byref(p), ctypes.byref(opts), _ptr(ws), ws.numel(),
                                 _stream(stream), ctypes.byref(res), G.ctypes.data_as(ctypes.c_void_p), host(al),
                                 host(be), host(F), host(st))
    _check(rc, "tnslq_logneg_dims")
    out: Dict[str, object] = res.as_dict()
    out["G"] = G[:res.n_probes_used].copy()
    if not loop:
        out.update({"alpha": al, "beta": be, "F": F, "steps": st})
    return out


def tnslq_rho_pt_dims(psi, dims, a, b, workspace=None, stream=None, out=None):
    """rho_AB^{T_B} in FP64 for a state on sites with dims[s] levels."""
    import numpy as np
    import torch
    _check_device_tensor(psi, "psi")
    dt = _dtype_code(psi)
    n = int(np.prod([dims[q] for q in list(a) + list(b)], dtype=np.int64))
    p = _partition_dims(dims, a, b)
    nb = ctypes.c_size_t(0)
    _check(lib().tnslq_rho_pt_dims_workspace_bytes(dt, ctypes.byref(p), ctypes.byref(nb)),
           "tnslq_rho_pt_dims_workspace_bytes")
    ws = _workspace(nb.value, psi.device, workspace)
    if out is None:
        out = torch.empty((n, n), dtype=torch.complex128, device=psi.device)
    _check(lib().tnslq_rho_pt_dims(_ptr(psi), dt, ctypes.byref(p), _ptr(out), _ptr(ws), ws.numel(), _stream(stream)),
           "tnslq_rho_pt_dims")
    return out


# ------------------------------------------------- matrix product states
def _mps_desc(tensors, tensors_ptr=None, sections="auto", matvec="auto"):
    """The library's description of an MPS (a list of (chi_l, p, chi_r)
    arrays; chi_l of the first = chi_r of the last, 1 for an open chain) with
    its tensors at ``tensors_ptr``; ``sections`` "auto", "explicit" or
    "transfer" (how compressed sections are formed), ``matvec`` "auto",
    "factors" or "network" (how the factorised route contracts a probe)."""
    if sections not in MPS_SECTIONS:
        raise ValueError(f"sections must be one of {sorted(MPS_SECTIONS)}, not {sections!r}")
    if matvec not in MPS_MATVEC:
        raise ValueError(f"matvec must be one of {sorted(MPS_MATVEC)}, not {matvec!r}")
    phys = [int(t.shape[1]) for t in tensors]
    bond = [int(tensors[0].shape[0])] + [int(t.shape[2]) for t in tensors]
    pp = (ctypes.c_int * len(phys))(*phys)
    bb = (ctypes.c_int * len(bond))(*bond)
    m = Mps(len(tensors), pp, bb, tensors_ptr, MPS_SECTIONS[sections], MPS_MATVEC[matvec])
    m._keep = (pp, bb)
    return m


def _mps(tensors, device, sections="auto", matvec="auto"):
    """Upload an MPS and describe it for the library."""
    import numpy as np
    import torch
    flat = np.concatenate([np.ascontiguousarray(np.asarray(t, dtype=np.complex128)).ravel() for t in tensors])
    dev = torch.from_numpy(flat).to(device)
    m = _mps_desc(tensors, _ptr(dev), sections, matvec)
    m._keep = m._keep + (dev,)
    return m


def tnslq_mps_effective_state(tensors, a0: int, n_a: int, b0: int, n_b: int, device="cuda", workspace=None,
                              stream=None, sections="auto"):
    """Sec. VI's compressed form of rho_AB^{T_B} for blocks A = [a0, a0 + n_a),
    B = [b0, b0 + n_b) of an open or periodic MPS, as a dense effective state:
    returns (psi_eff, (q_A, q_B, q_E)); psi_eff is a device complex128 vector
    of 2^(q_A + q_B + q_E) amplitudes, A' the most significant qubits."""
    import torch
    m = _mps(tensors, device, sections)
    q = (ctypes.c_int * 3)()
    n = ctypes.c_size_t(0)
    _check(lib().tnslq_mps_effective_state_size(ctypes.byref(m), int(a0), int(n_a), int(b0), int(n_b), q,
                                                ctypes.byref(n)), "tnslq_mps_effective_state_size")
    ws = _workspace(n.value, torch.device(device), workspace)
    psi = torch.empty(1 << (q[0] + q[1] + q[2]), dtype=torch.complex128, device=device)
    _check(lib().tnslq_mps_effective_state(ctypes.byref(m), int(a0), int(n_a), int(b0), int(n_b), _ptr(psi),
                                           _ptr(ws), ws.numel(), _stream(stream)), "tnslq_mps_effective_state")
    return psi, (q[0], q[1], q[2])


def tnslq_workspace_bytes_mps(tensors, a0: int, n_a: int, b0: int, n_b: int, opts: Options,
                              sections="auto", matvec="auto") -> int:
    m = _mps_desc(tensors, None, sections, matvec)
    n = ctypes.c_size_t(0)
    _check(lib().tnslq_workspace_bytes_mps(ctypes.byref(m), int(a0), int(n_a), int(b0), int(n_b), ctypes.byref(opts),
                                           ctypes.byref(n)), "tnslq_workspace_bytes_mps")
    return n.value


def tnslq_logneg_mps(tensors, a0: int, n_a: int, b0: int, n_b: int, n_probes: int, n_steps: int, device="cuda",
                     route="factored", reorth: bool = False, seed: int = 0, probe_offset: int = 0,
                     stop_tol: float = 0.0, stop_rule="diff", max_probes: int = 0, precision=None, workspace=None,
                     stream=None, want_arrays: bool = True, sections="auto", matvec="auto",
                     **kw) -> Dict[str, object]:
    """E(rho_AB) of two contiguous blocks of an open or periodic MPS (Sec. VI).

    route="factored": Algorithm 1 on the two-block operator in factorised form
    (tnslq_logneg_mps, precision "fp64" (default) or "fp32", nothing of the
    effective state's size formed); route="dense": the effective state of
    tnslq_mps_effective_state through tnslq_logneg in `precision` (its
    default when None; further keywords go to tnslq_logneg)."""
    import numpy as np
    import torch
    if route == "dense":
        psi, q = tnslq_mps_effective_state(tensors, a0, n_a, b0, n_b, device, sections=sections)
        qa, qb, qe = q
        if precision is not None:
            kw["precision"] = precision
        out = tnslq_logneg(psi, qa + qb + qe, list(range(qa)), list(range(qa, qa + qb)), n_probes, n_steps,
                           reorth=reorth, seed=seed, probe_offset=probe_offset, stop_tol=stop_tol,
                           stop_rule=stop_rule, max_probes=max_probes, want_arrays=want_arrays, **kw)
        out["effective_qubits"] = q
        return out
    if route != "factored":
        raise ValueError(f"route must be 'factored' or 'dense', not {route!r}")
    if kw:
        raise TypeError(f"unexpected keywords for the factored route: {sorted(kw)}")
    opts = make_options(n_probes, n_steps, reorth, precision or "fp64", seed, probe_offset, stop_tol, stop_rule,
                        "auto", max_probes)
    m = _mps(tensors, device, sections, matvec)
    need = tnslq_workspace_bytes_mps(tensors, a0, n_a, b0, n_b, opts, sections, matvec)
    ws = _workspace(need, torch.device(device), workspace)
    res = Result()
    loop = max_probes > n_probes
    K, s = n_probes, n_steps
    G = np.zeros(max_probes if loop else K)
    al, be, F = np.zeros((K, s)), np.zeros((K, s + 1)), np.zeros((K, s))
    st = np.zeros(K, dtype=np.int32)
    host = (lambda x: x.ctypes.data_as(ctypes.c_void_p)) if want_arrays and not loop else \
        (lambda x: ctypes.c_void_p(0))
    rc = lib().tnslq_logneg_mps(ctypes.byref(m), int(a0), int(n_a), int(b0), int(n_b), ctypes.byref(opts), _ptr(ws),
                                ws.numel(), _stream(stream), ctypes.byref(res), G.ctypes.data_as(ctypes.c_void_p),
                                host(al), host(be), host(F), host(st))
    _check(rc, "tnslq_logneg_mps")
    out: Dict[str, object] = res.as_dict()
    if loop:
        out["G"] = G[:res.n_probes_used].copy()
    elif want_arrays:
        out.update({"G": G, "alpha": al, "beta": be, "F": F, "steps": st})
    out["workspace_bytes"] = need
    return out


def tnslq_rho_pt_workspace_bytes(dtype: int, n_qubits: int, a, b) -> int:
    n = ctypes.c_size_t(0)
    p = _partition(n_qubits, a, b)
    _check(lib().tnslq_rho_pt_workspace_bytes(int(dtype), ctypes.byref(p), ctypes.byref(n)),
           "tnslq_rho_pt_workspace_bytes")
    return n.value


def tnslq_rho_pt(psi, n_qubits: int, a, b, workspace=None, stream=None, out=None):
    """rho_AB^{T_B} formed explicitly in FP64 (intermediary (iii)) as a device
    complex128 (d_A d_B, d_A d_B) matrix, rows and columns (a, b), b fastest."""
    import torch
    _check_device_tensor(psi, "psi")
    dt = _dtype_code(psi)
    n = 1 << (len(a) + len(b))
    need = tnslq_rho_pt_workspace_bytes(dt, n_qubits, a, b)
    ws = _workspace(need, psi.device, workspace)
    if out is None:
        out = torch.empty((n, n), dtype=torch.complex128, device=psi.device)
    p = _partition(n_qubits, a, b)
    _check(lib().tnslq_rho_pt(_ptr(psi), dt, ctypes.byref(p), _ptr(out), _ptr(ws), ws.numel(), _stream(stream)),
           "tnslq_rho_pt")
    return out


def tnslq_quadrature(alpha, beta, steps=None, stream=None):
    """Device FP64 (K, m) alpha, (K, m+1) beta -> (K, m) quadrature values."""
    import torch
    K, m = alpha.shape
    F = torch.empty((K, m), dtype=torch.float64, device=alpha.device)
    _check(lib().tnslq_quadrature(_ptr(alpha), _ptr(beta), _ptr(steps), K, m, _ptr(F), _stream(stream)),
           "tnslq_quadrature")
    return F


def tnslq_probes(seed: int, probe_offset: int, n_probes: int, d: int, device="cuda", stream=None):
    import torch
    X = torch.empty((n_probes, d), dtype=torch.complex128, device=device)
    _check(lib().tnslq_probes(int(seed) & (2**64 - 1), int(probe_offset), int(n_probes), int(d), _ptr(X),
                              _stream(stream)), "tnslq_probes")
    return X


# ------------------------------------------------------------- MLP
def tnslq_mlp_workspace_bytes(batch: int) -> int:
    n = ctypes.c_size_t(0)
    _check(lib().tnslq_mlp_workspace_bytes(int(batch), ctypes.byref(n)), "tnslq_mlp_workspace_bytes")
    return n.value


def tnslq_mlp_forward(params, norm, x, workspace=None, stream=None):
    import torch
    B = x.shape[0]
    out = torch.empty((B, MLP_NOUT), dtype=torch.float32, device=x.device)
    ws = _workspace(tnslq_mlp_workspace_bytes(B), x.device, workspace)
    _check(lib().tnslq_mlp_forward(_ptr(params), _ptr(norm), _ptr(x), B, _ptr(out), _ptr(ws), ws.numel(),
                                   _stream(stream)), "tnslq_mlp_forward")
    return out


def tnslq_mlp_loss_grad(params, norm, x, r, workspace=None, stream=None):
    import torch
    B = x.shape[0]
    loss = torch.empty(1, dtype=torch.float32, device=x.device)
    grad = torch.empty(MLP_NPARAMS, dtype=torch.float32, device=x.device)
    ws = _workspace(tnslq_mlp_workspace_bytes(B), x.device, workspace)
    _check(lib().tnslq_mlp_loss_grad(_ptr(params), _ptr(norm), _ptr(x), _ptr(r), B, _ptr(loss), _ptr(grad),
                                     _ptr(ws), ws.numel(), _stream(stream)), "tnslq_mlp_loss_grad")
    return loss, grad


def tnslq_mlp_adam(params, m, v, grad, t: int, lr: float, stream=None):
    _check(lib().tnslq_mlp_adam(_ptr(params), _ptr(m), _ptr(v), _ptr(grad), int(t), float(lr), _stream(stream)),
           "tnslq_mlp_adam")


def tnslq_mlp_train(params, m, v, norm, x, r, idx, batch: int, t0: int, lr: float, losses=None, workspace=None,
                    stream=None):
    n_batches = idx.numel() // batch
    need = tnslq_mlp_workspace_bytes(batch) + MLP_NPARAMS * 4 + 512
    ws = _workspace(need, x.device, workspace)
    _check(lib().tnslq_mlp_train(_ptr(params), _ptr(m), _ptr(v), _ptr(norm), _ptr(x), _ptr(r), _ptr(idx), int(batch),
                                 int(n_batches), int(t0), float(lr), _ptr(losses), _ptr(ws), ws.numel(),
                                 _stream(stream)), "tnslq_mlp_train")
    return t0 + n_batches


def tnslq_logneg_surrogate(psi, n_qubits: int, a, b, n_probes: int, n_steps: int, params, norm, y_scale: float,
                           tol: float = 0.01, early_steps: int = 8, reorth: bool = False, precision="fp32",
                           seed: int = 0, probe_offset: int = 0, stop_tol: float = 0.0, workspace=None,
                           stream=None, stop_rule="diff", operator="auto") -> Dict[str, object]:
    import numpy as np
    _check_device_tensor(psi, "psi")
    dt = _dtype_code(psi)
    opts = make_options(n_probes, n_steps, reorth, precision, seed, probe_offset, stop_tol, stop_rule, operator)
    p = _partition(n_qubits, a, b)
    need = tnslq_workspace_bytes(dt, n_qubits, a, b, opts)
    ws = _workspace(need, psi.device, workspace)
    res = Result()
    info = np.zeros(5)
    rc = lib().tnslq_logneg_surrogate(_ptr(psi), dt, ctypes.byref(p), ctypes.byref(opts), _ptr(params), _ptr(norm),
                                      float(y_scale), int(early_steps), float(tol), _ptr(ws), ws.numel(),
                                      _stream(stream), ctypes.byref(res), info.ctypes.data_as(ctypes.c_void_p))
    _check(rc, "tnslq_logneg_surrogate")
    out: Dict[str, object] = res.as_dict()
    out.update({"mu": info[0], "sigma": info[1], "e_early": info[2], "used_fallback": bool(info[3]),
                "e_full": info[4] if not math.isnan(info[4]) else None})
    return out


# ------------------------------------------------------------- entropy
def _qubits(s: Sequence[int]):
    arr = (ctypes.c_int * max(1, len(s)))(*s)
    return arr


def tnslq_spectral_workspace_bytes(dtype: int, n_qubits: int, s, opts: Options) -> int:
    n = ctypes.c_size_t(0)
    arr = _qubits(s)
    _check(lib().tnslq_spectral_workspace_bytes(int(dtype), int(n_qubits), ctypes.cast(arr, ctypes.c_void_p), len(s),
                                                ctypes.byref(opts), ctypes.byref(n)), "tnslq_spectral_workspace_bytes")
    return n.value


def tnslq_spectral_sum(psi, n_qubits: int, s, fn="entropy", n_probes: int = 8, n_steps: int = 40,
                       reorth: bool = False, seed: int = 0, probe_offset: int = 0, workspace=None, stream=None,
                       want_arrays: bool = True) -> Dict[str, object]:
    """Tr f(rho_S) of the device state ``psi`` for f = -x log2 x ("entropy") or x^2 ("purity")."""
    import numpy as np
    _check_device_tensor(psi, "psi")
    if psi.numel() != 1 << n_qubits:
        raise ValueError("psi has the wrong length")
    dt = _dtype_code(psi)
    code = FUNCTIONS[fn] if isinstance(fn, str) else int(fn)
    opts = make_options(n_probes, n_steps, reorth, "fp64", seed, probe_offset, 0.0)
    need = tnslq_spectral_workspace_bytes(dt, n_qubits, s, opts)
    ws = _workspace(max(need, 256), psi.device, workspace)
    res = SpectralResult()
    K, m = n_probes, n_steps
    G = np.zeros(K)
    al = np.zeros((K, m))
    be = np.zeros((K, m + 1))
    F = np.zeros((K, m))
    st = np.zeros(K, dtype=np.int32)
    host = (lambda x: x.ctypes.data_as(ctypes.c_void_p)) if want_arrays else (lambda x: ctypes.c_void_p(0))
    arr = _qubits(s)
    rc = lib().tnslq_spectral_sum(_ptr(psi), dt, int(n_qubits), ctypes.cast(arr, ctypes.c_void_p), len(s), code,
                                  ctypes.byref(opts), _ptr(ws), ws.numel(), _stream(stream), ctypes.byref(res),
                                  host(G), host(al), host(be), host(F), host(st))
    _check(rc, "tnslq_spectral_sum")
    out: Dict[str, object] = res.as_dict()
    if want_arrays:
        out.update({"G": G, "alpha": al, "beta": be, "F": F, "steps": st})
    return out


def tnslq_mutual_information(psi, n_qubits: int, a, b, n_probes: int = 8, n_steps: int = 40, reorth: bool = False,
                             seed: int = 0, probe_offset: int = 0, workspace=None, stream=None) -> Dict[str, float]:
    """I(A:B) = S(A) + S(B) - S(AB) of the device state ``psi``, in bits."""
    import numpy as np
    _check_device_tensor(psi, "psi")
    dt = _dtype_code(psi)
    opts = make_options(n_probes, n_steps, reorth, "fp64", seed, probe_offset, 0.0)
    p = _partition(n_qubits, a, b)
    n = ctypes.c_size_t(0)
    _check(lib().tnslq_mutual_information_workspace_bytes(dt, ctypes.byref(p), ctypes.byref(opts), ctypes.byref(n)),
           "tnslq_mutual_information_workspace_bytes")
    ws = _workspace(max(n.value, 256), psi.device, workspace)
    out = np.zeros(8)
    _check(lib().tnslq_mutual_information(_ptr(psi), dt, ctypes.byref(p), ctypes.byref(opts), _ptr(ws), ws.numel(),
                                          _stream(stream), out.ctypes.data_as(ctypes.c_void_p)),
           "tnslq_mutual_information")
    keys = ("mutual_information", "mutual_information_se", "S_A", "S_A_se", "S_B", "S_B_se", "S_AB", "S_AB_se")
    return {k: float(v) for k, v in zip(keys, out)}
