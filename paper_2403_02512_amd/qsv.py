"""ctypes binding of libqsv (include/qsv.h): argument marshalling only.

Every step of the hot path runs in the HIP library; this module converts
Python circuit descriptions (``workloads.Op`` / ``workloads.PauliSum``) into
the C structs, hands over device pointers (torch tensors or library-owned
buffers) and raises ``QsvError`` on a non-zero status.  There is no CPU
fallback: without the built library or a GPU the calls fail loudly.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import sys
import weakref
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# QSV_LIB_PATH: load another build of the library (the CPU suite's
# sanitizer build); the default is the in-tree libqsv.so
LIB_PATH = os.environ.get("QSV_LIB_PATH") or os.path.join(_HERE, "libqsv.so")

C64, C128 = 1, 2
MAX_QUBITS = 34
ADJ_INPLACE = 1
OPT_FUSION, OPT_TILE_BITS, OPT_TILE_BITS_ADJ, OPT_LOW_BITS, OPT_PROFILE, OPT_NONTEMPORAL, OPT_LAYERS = 1, 2, 3, 4, 5, 6, 7
OPT_TEST_ALLOC_LIMIT, OPT_TEST_FAIL_LAUNCH = 8, 9   # fault injection (tests of the error paths)
OPT_TILE_WS, OPT_DENSE_MFMA = 10, 11

GATE_IDS = {
    "PauliX": 1, "PauliY": 2, "PauliZ": 3, "Hadamard": 4, "S": 5, "T": 6, "SX": 7, "Identity": 8,
    "PhaseShift": 20, "RX": 21, "RY": 22, "RZ": 23, "Rot": 24, "U3": 25,
    "CNOT": 40, "CY": 41, "CZ": 42, "SWAP": 43, "CRX": 44, "CRY": 45, "CRZ": 46, "CRot": 47,
    "ControlledPhaseShift": 48, "IsingXX": 49, "IsingYY": 50, "IsingZZ": 51, "IsingXY": 52,
    "SingleExcitation": 53, "Toffoli": 70, "CSWAP": 71, "DoubleExcitation": 72, "MultiRZ": 73,
    "QubitUnitary": 90,
}

STATUS = {0: "ok", -1: "invalid argument", -2: "invalid wire", -3: "dtype mismatch", -4: "out of memory",
          -5: "HIP runtime error", -6: "unsupported", -7: "invalid parameter index"}


class QsvError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"qsv status {status} ({STATUS.get(status, '?')}): {msg}")
        self.status = status


class QsvOp(ctypes.Structure):
    _fields_ = [("gate", ctypes.c_int32), ("n_wires", ctypes.c_int32), ("n_ctrls", ctypes.c_int32),
                ("ctrl_values", ctypes.c_uint32), ("inverse", ctypes.c_int32), ("wires", ctypes.c_int32 * 8),
                ("param", ctypes.c_int32 * 3), ("scale", ctypes.c_double * 3), ("matrix_offset", ctypes.c_int64)]


class QsvPauliSum(ctypes.Structure):
    _fields_ = [("n_terms", ctypes.c_int64), ("coeff", ctypes.POINTER(ctypes.c_double)),
                ("x_mask", ctypes.POINTER(ctypes.c_uint64)), ("z_mask", ctypes.POINTER(ctypes.c_uint64))]


_lib = None
_live = weakref.WeakSet()   # contexts and states still open, released before interpreter exit


def _close_all():
    objs = list(_live)
    for o in objs:              # states and batches first: they belong to contexts
        if not isinstance(o, Context):
            o.close()
    for o in objs:
        if isinstance(o, Context):
            o.close()


atexit.register(_close_all)

EXPORTS = [
    "qsv_version", "qsv_status_string", "qsv_thread_last_error", "qsv_device_count", "qsv_ctx_create",
    "qsv_ctx_destroy", "qsv_last_error", "qsv_ctx_set_stream", "qsv_ctx_synchronize", "qsv_ctx_set_option",
    "qsv_ctx_get_option", "qsv_ctx_workspace_bytes", "qsv_ctx_release_workspace", "qsv_kernel_kinds",
    "qsv_kernel_name", "qsv_ctx_kernel_stats", "qsv_ctx_reset_stats", "qsv_state_create", "qsv_state_wrap",
    "qsv_state_destroy", "qsv_state_n_qubits", "qsv_state_device_ptr", "qsv_state_reset", "qsv_state_copy",
    "qsv_state_to_host", "qsv_state_from_host", "qsv_validate_ops", "qsv_validate_obs", "qsv_apply",
    "qsv_expval", "qsv_expval_noalloc", "qsv_adjoint_jacobian", "qsv_adjoint_vjp", "qsv_plan_stats", "qsv_plan_json", "qsv_var",
    "qsv_probs", "qsv_expval_sparse", "qsv_batch_create", "qsv_batch_destroy", "qsv_batch_run", "qsv_sample",
    "qsv_autotune",
]


def lib():
    """Load libqsv.so (built by paper_2403_02512_amd.build); raise if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2403_02512_amd.build`")
    # PyTorch ships its own HIP runtime library; loading it first lets this
    # library bind to the same one, so that one runtime serves the process
    # (with two, whichever initialises second can find no devices)
    if not os.environ.get("QSV_LIB_PATH"):
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, u32, u64, dp = (ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64,
                                 ctypes.POINTER(ctypes.c_double))
    sz = ctypes.c_size_t
    opp = ctypes.POINTER(QsvOp)
    obp = ctypes.POINTER(QsvPauliSum)
    sig = {
        "qsv_version": ([], ctypes.c_char_p), "qsv_status_string": ([i32], ctypes.c_char_p),
        "qsv_thread_last_error": ([], ctypes.c_char_p), "qsv_device_count": ([], i32),
        "qsv_ctx_create": ([i32, vp, ctypes.POINTER(vp)], i32), "qsv_ctx_destroy": ([vp], None),
        "qsv_last_error": ([vp], ctypes.c_char_p), "qsv_ctx_set_stream": ([vp, vp], i32),
        "qsv_ctx_synchronize": ([vp], i32), "qsv_ctx_set_option": ([vp, i32, i64], i32),
        "qsv_ctx_get_option": ([vp, i32, ctypes.POINTER(i64)], i32),
        "qsv_ctx_workspace_bytes": ([vp, ctypes.POINTER(sz)], i32), "qsv_ctx_release_workspace": ([vp], i32),
        "qsv_kernel_kinds": ([], i32), "qsv_kernel_name": ([i32], ctypes.c_char_p),
        "qsv_ctx_kernel_stats": ([vp, i32, ctypes.POINTER(i64), dp, dp], i32), "qsv_ctx_reset_stats": ([vp], i32),
        "qsv_state_create": ([vp, i32, i32, ctypes.POINTER(vp)], i32),
        "qsv_state_wrap": ([vp, i32, i32, vp, ctypes.POINTER(vp)], i32), "qsv_state_destroy": ([vp], None),
        "qsv_state_n_qubits": ([vp], i32), "qsv_state_device_ptr": ([vp], vp),
        "qsv_state_reset": ([vp, u64], i32), "qsv_state_copy": ([vp, vp], i32),
        "qsv_state_to_host": ([vp, vp], i32), "qsv_state_from_host": ([vp, vp], i32),
        "qsv_validate_ops": ([i32, opp, sz, sz, sz], i32), "qsv_validate_obs": ([i32, obp, sz], i32),
        "qsv_apply": ([vp, opp, sz, dp, sz, dp, sz], i32),
        "qsv_expval": ([vp, obp, sz, dp], i32),
        "qsv_expval_noalloc": ([vp, obp, sz, dp], i32),
        "qsv_var": ([vp, obp, sz, dp], i32),
        "qsv_probs": ([vp, ctypes.POINTER(ctypes.c_int32), i32, dp], i32),
        "qsv_expval_sparse": ([vp, ctypes.POINTER(i64), ctypes.POINTER(i64), dp, i64, dp], i32),
        "qsv_adjoint_jacobian": ([vp, opp, sz, dp, sz, dp, sz, obp, sz, dp, dp, u32], i32),
        "qsv_adjoint_vjp": ([vp, opp, sz, dp, sz, dp, sz, obp, sz, dp, dp, dp, u32], i32),
        "qsv_plan_stats": ([i32, i32, opp, sz, dp, sz, dp, sz, i32, i32, i32, i32, ctypes.POINTER(i64),
                            ctypes.POINTER(i64), ctypes.POINTER(i64), dp], i32),
        "qsv_plan_json": ([i32, i32, opp, sz, dp, sz, dp, sz, i32, i32, i32, i32, ctypes.c_char_p, sz,
                           ctypes.POINTER(sz)], i32),
        "qsv_batch_create": ([vp, i32, sz, ctypes.POINTER(ctypes.c_int32), opp, ctypes.POINTER(sz),
                              ctypes.POINTER(sz), dp, sz, obp, ctypes.POINTER(vp)], i32),
        "qsv_batch_destroy": ([vp], None),
        "qsv_batch_run": ([vp, dp, dp, dp, u32], i32),
        "qsv_sample": ([vp, dp, sz, ctypes.POINTER(u64)], i32),
        "qsv_autotune": ([vp, opp, sz, dp, sz, dp, sz, obp, sz, ctypes.POINTER(ctypes.c_int32),
                          ctypes.POINTER(ctypes.c_int32)], i32),
    }
    for name in EXPORTS:
        f = getattr(L, name)
        f.argtypes, f.restype = sig[name]
    _lib = L
    return L


def _check(status: int, ctx=None):
    if status != 0:
        L = lib()
        msg = (L.qsv_last_error(ctx) if ctx else L.qsv_thread_last_error()) or b""
        raise QsvError(status, msg.decode(errors="replace"))


def _dptr(a: Optional[np.ndarray]):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


# ------------------------------------------------------------------ marshalling

class MarshalledOps:
    """C op array plus the matrices and parameters it refers to (kept alive)."""

    def __init__(self, ops, params):
        n = len(ops)
        self.arr = (QsvOp * max(1, n))()
        mats = []
        moff = 0
        for i, op in enumerate(ops):
            o = self.arr[i]
            o.gate = GATE_IDS[op.name]
            o.n_wires = len(op.wires)
            o.n_ctrls = op.n_ctrls
            o.ctrl_values = (op.ctrl_values if op.ctrl_values >= 0 else (1 << op.n_ctrls) - 1) & 0xFFFFFFFF
            o.inverse = int(bool(op.inverse))
            for j, w in enumerate(op.wires):
                o.wires[j] = w
            for s in range(3):
                o.param[s] = op.param[s] if s < len(op.param) else -1
                o.scale[s] = op.scale[s] if s < len(op.scale) else 0.0
            if op.matrix is not None:
                m = np.ascontiguousarray(op.matrix, dtype=np.complex128).ravel()
                o.matrix_offset = moff
                mats.append(m)
                moff += m.size
            else:
                o.matrix_offset = -1
        self.n = n
        self.matrices = np.concatenate(mats) if mats else np.zeros(1, dtype=np.complex128)
        self.n_mat = moff
        self.params = np.ascontiguousarray(params if params is not None else np.zeros(0), dtype=np.float64).reshape(-1)
        self.n_params = self.params.size
        if self.params.size == 0:
            self.params = np.zeros(1)

    def mat_ptr(self):
        return self.matrices.view(np.float64).ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def pauli_masks(word: str):
    """(x_mask, z_mask) of a Pauli word given per wire (wire 0 = msb)."""
    n = len(word)
    x = z = 0
    for w, l in enumerate(word):
        bit = 1 << (n - 1 - w)
        if l in "XY":
            x |= bit
        if l in "ZY":
            z |= bit
        if l not in "IXYZ":
            raise ValueError(f"bad Pauli letter {l!r}")
    return x, z


class MarshalledObs:
    def __init__(self, observables):
        self.keep = []
        self.arr = (QsvPauliSum * max(1, len(observables)))()
        for i, o in enumerate(observables):
            c = np.ascontiguousarray(o.coeffs, dtype=np.float64)
            xs = np.zeros(len(o.words), dtype=np.uint64)
            zs = np.zeros(len(o.words), dtype=np.uint64)
            for t, w in enumerate(o.words):
                xs[t], zs[t] = pauli_masks(w)
            self.keep += [c, xs, zs]
            h = self.arr[i]
            h.n_terms = len(o.words)
            h.coeff = c.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
            h.x_mask = xs.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))
            h.z_mask = zs.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))
        self.n = len(observables)


def validate_ops(n_qubits: int, ops, n_params: int) -> None:
    """Host-only validation of an op list (no device needed)."""
    m = MarshalledOps(ops, np.zeros(n_params))
    _check(lib().qsv_validate_ops(n_qubits, m.arr, m.n, n_params, m.n_mat))


def validate_obs(n_qubits: int, observables) -> None:
    m = MarshalledObs(observables)
    _check(lib().qsv_validate_obs(n_qubits, m.arr, m.n))


def plan_stats(n_qubits: int, ops, params, dtype: int = C128, adjoint: bool = False, tile_bits: int = 0,
               low_bits: int = 0, fusion: bool = True) -> dict:
    """Host-only plan summary: passes over the state, tiled passes, lowered
    tile ops and algorithmic HBM bytes (no device needed)."""
    m = MarshalledOps(ops, params)
    a, b, c = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    by = ctypes.c_double()
    _check(lib().qsv_plan_stats(n_qubits, dtype, m.arr, m.n, _dptr(m.params), m.n_params, m.mat_ptr(), m.n_mat,
                                int(adjoint), tile_bits, low_bits, int(fusion), ctypes.byref(a), ctypes.byref(b),
                                ctypes.byref(c), ctypes.byref(by)))
    return {"passes": a.value, "tile_passes": b.value, "kernel_ops": c.value, "alg_bytes": by.value}


def plan_json(n_qubits: int, ops, params, dtype: int = C128, adjoint: bool = False, tile_bits: int = 0,
              low_bits: int = 0, fusion: bool = True) -> dict:
    """Host-only dump of the lowered program (passes, tile ops, tables)."""
    import json
    m = MarshalledOps(ops, params)
    need = ctypes.c_size_t()
    args = (n_qubits, dtype, m.arr, m.n, _dptr(m.params), m.n_params, m.mat_ptr(), m.n_mat, int(adjoint),
            tile_bits, low_bits, int(fusion))
    _check(lib().qsv_plan_json(*args, None, 0, ctypes.byref(need)))
    buf = ctypes.create_string_buffer(need.value)
    _check(lib().qsv_plan_json(*args, buf, need.value, ctypes.byref(need)))
    return json.loads(buf.value.decode())


def device_count() -> int:
    return int(lib().qsv_device_count())


# ------------------------------------------------------------------ context / state

class Context:
    """One device and one HIP stream.  stream: an int hipStream_t handle
    (e.g. ``torch.cuda.current_stream().cuda_stream``) or None for an owned
    stream."""

    def __init__(self, device: int = 0, stream: Optional[int] = None):
        L = lib()
        h = ctypes.c_void_p()
        _check(L.qsv_ctx_create(device, ctypes.c_void_p(stream) if stream else None, ctypes.byref(h)))
        self.h = h
        self.device = device
        self.states = weakref.WeakSet()
        _live.add(self)

    def close(self):
        if getattr(self, "h", None):
            for st in list(self.states):   # a state must not outlive its context
                st.close()
            lib().qsv_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        if sys.is_finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    def set_stream(self, stream: Optional[int]):
        _check(lib().qsv_ctx_set_stream(self.h, ctypes.c_void_p(stream) if stream else None), self.h)

    def synchronize(self):
        _check(lib().qsv_ctx_synchronize(self.h), self.h)

    def set_option(self, opt: int, value: int):
        _check(lib().qsv_ctx_set_option(self.h, opt, int(value)), self.h)

    def get_option(self, opt: int) -> int:
        v = ctypes.c_int64()
        _check(lib().qsv_ctx_get_option(self.h, opt, ctypes.byref(v)), self.h)
        return v.value

    def workspace_bytes(self) -> int:
        v = ctypes.c_size_t()
        _check(lib().qsv_ctx_workspace_bytes(self.h, ctypes.byref(v)), self.h)
        return v.value

    def release_workspace(self):
        _check(lib().qsv_ctx_release_workspace(self.h), self.h)

    def kernel_stats(self) -> dict:
        L = lib()
        out = {}
        for k in range(L.qsv_kernel_kinds()):
            n = ctypes.c_int64()
            ms = ctypes.c_double()
            by = ctypes.c_double()
            _check(L.qsv_ctx_kernel_stats(self.h, k, ctypes.byref(n), ctypes.byref(ms), ctypes.byref(by)), self.h)
            if n.value:
                out[L.qsv_kernel_name(k).decode()] = {"launches": n.value, "ms": ms.value, "bytes": by.value}
        return out

    def reset_stats(self):
        _check(lib().qsv_ctx_reset_stats(self.h), self.h)


class State:
    """2^n amplitudes in device memory: owned (allocated by the library) or
    wrapping a torch tensor (complex128 / complex64, contiguous, on the
    context's device), which the state keeps alive."""

    def __init__(self, ctx: Context, n_qubits: int, dtype: int = C128, tensor=None):
        L = lib()
        h = ctypes.c_void_p()
        self.ctx = ctx
        self.n = n_qubits
        self.dtype = dtype
        self.tensor = tensor
        if tensor is not None:
            import torch
            want = torch.complex128 if dtype == C128 else torch.complex64
            if tensor.dtype != want or not tensor.is_contiguous() or tensor.numel() != (1 << n_qubits):
                raise ValueError("tensor must be a contiguous 2^n complex tensor of the state's dtype")
            _check(L.qsv_state_wrap(ctx.h, n_qubits, dtype, ctypes.c_void_p(tensor.data_ptr()), ctypes.byref(h)),
                   ctx.h)
        else:
            _check(L.qsv_state_create(ctx.h, n_qubits, dtype, ctypes.byref(h)), ctx.h)
        self.h = h
        _live.add(self)
        ctx.states.add(self)

    def close(self):
        if getattr(self, "h", None) and getattr(self.ctx, "h", None):
            lib().qsv_state_destroy(self.h)
        self.h = None

    def __del__(self):
        if sys.is_finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    @property
    def np_dtype(self):
        return np.complex128 if self.dtype == C128 else np.complex64

    def reset(self, basis: int = 0):
        _check(lib().qsv_state_reset(self.h, basis), self.ctx.h)

    def copy_from(self, other: "State"):
        _check(lib().qsv_state_copy(self.h, other.h), self.ctx.h)

    def to_numpy(self) -> np.ndarray:
        out = np.empty(1 << self.n, dtype=self.np_dtype)
        _check(lib().qsv_state_to_host(self.h, out.ctypes.data_as(ctypes.c_void_p)), self.ctx.h)
        return out

    def from_numpy(self, a: np.ndarray):
        a = np.ascontiguousarray(a, dtype=self.np_dtype)
        if a.size != 1 << self.n:
            raise ValueError("size mismatch")
        _check(lib().qsv_state_from_host(self.h, a.ctypes.data_as(ctypes.c_void_p)), self.ctx.h)


# ------------------------------------------------------------------ hot path

def apply(state: State, ops, params=None, marshalled: Optional[MarshalledOps] = None) -> None:
    m = marshalled or MarshalledOps(ops, params)
    _check(lib().qsv_apply(state.h, m.arr, m.n, _dptr(m.params), m.n_params, m.mat_ptr(), m.n_mat), state.ctx.h)


def expval(state: State, observables, marshalled: Optional[MarshalledObs] = None) -> np.ndarray:
    mo = marshalled or MarshalledObs(observables)
    out = np.zeros(max(1, mo.n))
    _check(lib().qsv_expval(state.h, mo.arr, mo.n, _dptr(out)), state.ctx.h)
    return out[: mo.n]


def expval_noalloc(state: State, observables, marshalled: Optional[MarshalledObs] = None) -> np.ndarray:
    """qsv_expval_noalloc: expval with no device allocation (static scratch)."""
    mo = marshalled or MarshalledObs(observables)
    out = np.zeros(max(1, mo.n))
    _check(lib().qsv_expval_noalloc(state.h, mo.arr, mo.n, _dptr(out)), state.ctx.h)
    return out[: mo.n]


def var(state: State, observables, marshalled: Optional[MarshalledObs] = None) -> np.ndarray:
    mo = marshalled or MarshalledObs(observables)
    out = np.zeros(max(1, mo.n))
    _check(lib().qsv_var(state.h, mo.arr, mo.n, _dptr(out)), state.ctx.h)
    return out[: mo.n]


def expval_sparse(state: State, matrix) -> complex:
    """<psi|S|psi> for a scipy.sparse matrix S (converted to CSR, complex128)."""
    import scipy.sparse as sp
    m = sp.csr_matrix(matrix, dtype=np.complex128)
    m.sort_indices()
    rp = np.ascontiguousarray(m.indptr, dtype=np.int64)
    ci = np.ascontiguousarray(m.indices, dtype=np.int64)
    va = np.ascontiguousarray(m.data, dtype=np.complex128).view(np.float64)
    out = np.zeros(2)
    i64p = ctypes.POINTER(ctypes.c_int64)
    _check(lib().qsv_expval_sparse(state.h, rp.ctypes.data_as(i64p), ci.ctypes.data_as(i64p), _dptr(va), m.nnz,
                                   _dptr(out)), state.ctx.h)
    return complex(out[0], out[1])


def probs(state: State, wires: Sequence[int]) -> np.ndarray:
    """Marginal probabilities of the listed wires (first wire = msb)."""
    w = np.ascontiguousarray(wires, dtype=np.int32)
    out = np.zeros(1 << len(w))
    _check(lib().qsv_probs(state.h, w.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), len(w), _dptr(out)),
           state.ctx.h)
    return out


def autotune(state: State, ops, params, observables=()) -> tuple:
    """Time the circuit (and its adjoint, if observables are given) for each
    LDS tile width, set the fastest on the context; -> (tile_bits,
    tile_bits_adj).  Overwrites the state with the circuit's output."""
    m = MarshalledOps(ops, params)
    mo = MarshalledObs(list(observables))
    a, b = ctypes.c_int32(), ctypes.c_int32()
    _check(lib().qsv_autotune(state.h, m.arr, m.n, _dptr(m.params), m.n_params, m.mat_ptr(), m.n_mat, mo.arr, mo.n,
                              ctypes.byref(a), ctypes.byref(b)), state.ctx.h)
    return a.value, b.value


def sample(state: State, u) -> np.ndarray:
    """Basis indices drawn from |psi|^2 by inverse transform of the caller's
    uniforms u in [0, 1)."""
    u = np.ascontiguousarray(u, dtype=np.float64).reshape(-1)
    out = np.zeros(max(1, u.size), dtype=np.uint64)
    _check(lib().qsv_sample(state.h, _dptr(u if u.size else np.zeros(1)), u.size,
                            out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))), state.ctx.h)
    return out[:u.size].astype(np.int64)


def adjoint_jacobian(state: State, ops, params, observables, inplace: bool = False,
                     marshalled: Optional[MarshalledOps] = None, marshalled_obs: Optional[MarshalledObs] = None):
    """(jac[n_obs, n_params], expvals[n_obs]) from the post-circuit state."""
    m = marshalled or MarshalledOps(ops, params)
    mo = marshalled_obs or MarshalledObs(observables)
    jac = np.zeros((max(1, mo.n), max(1, m.n_params)))
    ev = np.zeros(max(1, mo.n))
    _check(lib().qsv_adjoint_jacobian(state.h, m.arr, m.n, _dptr(m.params), m.n_params, m.mat_ptr(), m.n_mat,
                                      mo.arr, mo.n, _dptr(jac), _dptr(ev), ADJ_INPLACE if inplace else 0),
           state.ctx.h)
    return jac[: mo.n, : m.n_params], ev[: mo.n]


def adjoint_vjp(state: State, ops, params, observables, cotangent: Sequence[float], inplace: bool = False,
                want_expval: bool = True, marshalled: Optional[MarshalledOps] = None,
                marshalled_obs: Optional[MarshalledObs] = None):
    """(grad[n_params], expvals[n_obs]) with grad = sum_o cot_o d<H_o>/dparams."""
    m = marshalled or MarshalledOps(ops, params)
    mo = marshalled_obs or MarshalledObs(observables)
    cot = np.ascontiguousarray(cotangent, dtype=np.float64)
    if cot.size != mo.n:
        raise ValueError("one cotangent per observable")
    grad = np.zeros(max(1, m.n_params))
    ev = np.zeros(max(1, mo.n))
    _check(lib().qsv_adjoint_vjp(state.h, m.arr, m.n, _dptr(m.params), m.n_params, m.mat_ptr(), m.n_mat, mo.arr,
                                 mo.n, _dptr(cot), _dptr(grad), _dptr(ev) if want_expval else None,
                                 ADJ_INPLACE if inplace else 0), state.ctx.h)
    return grad[: m.n_params], ev[: mo.n]


# ------------------------------------------------------------------ batches

BATCH_GRAPH = 1


class Batch:
    """Independent circuits (each with one observable, possibly of different
    widths) run together: pass s of every circuit shares one launch, and with
    ``graph=True`` the launch sequence is captured once in a HIP graph and
    replayed for new parameters.  circuits: objects with n_qubits, ops,
    n_params and observables (the first is used)."""

    def __init__(self, ctx: Context, circuits, dtype: int = C128):
        self.ctx = ctx
        self.dtype = dtype
        self.n_circuits = len(circuits)
        self.n_params = [int(c.n_params) for c in circuits]
        self.p_off = np.concatenate([[0], np.cumsum(self.n_params)]).astype(np.int64)
        ms = [MarshalledOps(c.ops, np.zeros(c.n_params)) for c in circuits]
        n_ops = sum(m.n for m in ms)
        self._ops = (QsvOp * max(1, n_ops))()
        offs = np.zeros(self.n_circuits + 1, dtype=np.uintp)
        mats, moff, k = [], 0, 0
        for i, m in enumerate(ms):
            offs[i] = k
            for j in range(m.n):
                o = m.arr[j]
                if o.matrix_offset >= 0:
                    o.matrix_offset += moff
                self._ops[k] = o
                k += 1
            if m.n_mat:
                mats.append(m.matrices[:m.n_mat])
                moff += m.n_mat
        offs[-1] = k
        self._mats = np.concatenate(mats) if mats else np.zeros(1, dtype=np.complex128)
        self._obs = MarshalledObs([c.observables[0] for c in circuits])
        nq = np.array([c.n_qubits for c in circuits], dtype=np.int32)
        npar = np.array(self.n_params, dtype=np.uintp)
        h = ctypes.c_void_p()
        L = lib()
        _check(L.qsv_batch_create(ctx.h, dtype, self.n_circuits, nq.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                  self._ops, offs.ctypes.data_as(ctypes.POINTER(ctypes.c_size_t)),
                                  npar.ctypes.data_as(ctypes.POINTER(ctypes.c_size_t)),
                                  self._mats.view(np.float64).ctypes.data_as(ctypes.POINTER(ctypes.c_double)), moff,
                                  self._obs.arr, ctypes.byref(h)), ctx.h)
        self.h = h
        ctx.states.add(self)
        _live.add(self)

    def close(self):
        if getattr(self, "h", None):
            lib().qsv_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        if sys.is_finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    def run(self, params, grad: bool = True, graph: bool = False):
        """-> (expvals [n_circuits], list of per-circuit gradients or None)."""
        p = np.ascontiguousarray(np.concatenate([np.asarray(x, dtype=np.float64).reshape(-1) for x in params])
                                 if len(params) else np.zeros(0), dtype=np.float64)
        if p.size != self.p_off[-1]:
            raise ValueError(f"expected {self.p_off[-1]} parameters in total, got {p.size}")
        ev = np.zeros(self.n_circuits)
        g = np.zeros(max(1, p.size)) if grad else None
        _check(lib().qsv_batch_run(self.h, _dptr(p if p.size else np.zeros(1)), _dptr(ev), _dptr(g),
                                   BATCH_GRAPH if graph else 0), self.ctx.h)
        if not grad:
            return ev, None
        return ev, [g[self.p_off[i]:self.p_off[i + 1]].copy() for i in range(self.n_circuits)]
