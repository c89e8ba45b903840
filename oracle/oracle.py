"""ctypes front-end of the plain FP64 CPU oracle (``oracle.c``).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark are the only users.  Nothing in the GPU library imports
this module and this module imports nothing from the GPU library.

Circuits come in as plain Python objects with the attributes
``name, wires, param, scale, inverse, n_ctrls, ctrl_values, matrix``
(one per operation); observables as objects with ``coeffs`` and ``words``
(one Pauli letter per wire, wire 0 first).  Wire 0 is the most significant
index bit (paper Sec. 2.1.1, Alg. 1).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
# ORACLE_LIB_PATH: load another build of the oracle (the CPU suite's
# sanitizer build); the default is the in-tree liboracle.so
_LIB_PATH = os.environ.get("ORACLE_LIB_PATH") or os.path.join(_HERE, "liboracle.so")

# Gate numbering of oracle.h (enum orc_gate), keyed by PennyLane gate names.
GATES = {
    "Identity": 0, "PauliX": 1, "PauliY": 2, "PauliZ": 3, "Hadamard": 4, "S": 5, "T": 6, "SX": 7,
    "PhaseShift": 8, "RX": 9, "RY": 10, "RZ": 11, "Rot": 12, "U3": 13,
    "CNOT": 14, "CY": 15, "CZ": 16, "SWAP": 17,
    "CRX": 18, "CRY": 19, "CRZ": 20, "CRot": 21, "ControlledPhaseShift": 22,
    "IsingXX": 23, "IsingYY": 24, "IsingZZ": 25, "IsingXY": 26, "SingleExcitation": 27,
    "Toffoli": 28, "CSWAP": 29, "DoubleExcitation": 30, "MultiRZ": 31, "QubitUnitary": 32,
}


class OrcOp(ctypes.Structure):
    _fields_ = [
        ("gate", ctypes.c_int32), ("n_wires", ctypes.c_int32), ("n_ctrls", ctypes.c_int32),
        ("ctrl_values", ctypes.c_uint32), ("inverse", ctypes.c_int32),
        ("wires", ctypes.c_int32 * 8), ("param", ctypes.c_int32 * 3),
        ("scale", ctypes.c_double * 3), ("matrix_offset", ctypes.c_int64),
    ]


def build(force: bool = False) -> str:
    """Compile liboracle.so next to its source (plain C, -O2, no FMA contraction)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call([
            "gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
            "-std=gnu11", "-Wall", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def build_sanitized(out_dir: str) -> str:
    """Compile the oracle with AddressSanitizer and UndefinedBehaviorSanitizer
    (any report aborts) into out_dir; used by the CPU suite's sanitizer run."""
    os.makedirs(out_dir, exist_ok=True)
    out = os.path.join(out_dir, "liboracle.so")
    subprocess.check_call([
        "gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
        "-fno-sanitize-recover=undefined", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
        "-std=gnu11", "-Wall", _SRC, "-o", out, "-lm"])
    return out


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.environ.get("ORACLE_LIB_PATH"):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        i32p = ctypes.POINTER(ctypes.c_int32)
        L.orc_gate_matrix.argtypes = [ctypes.c_int, ctypes.c_int, dp, ctypes.c_int, dp]
        L.orc_gate_generator.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp]
        L.orc_apply_matrix.argtypes = [ctypes.c_int, dp, ctypes.c_int, i32p, dp]
        L.orc_apply_matrix.restype = None
        L.orc_apply.argtypes = [ctypes.c_int, dp, ctypes.POINTER(OrcOp), ctypes.c_int64, dp, dp]
        L.orc_inner.argtypes = [ctypes.c_int, dp, dp, dp]
        L.orc_inner.restype = None
        L.orc_expval.argtypes = [ctypes.c_int, dp, ctypes.c_int, i32p, dp, ctypes.c_char_p, dp]
        L.orc_apply_pauli_sum.argtypes = [ctypes.c_int, dp, ctypes.c_int, dp, ctypes.c_char_p, dp]
        L.orc_sample.argtypes = [ctypes.c_int, dp, ctypes.c_int64, dp, ctypes.POINTER(ctypes.c_int64)]
        L.orc_adjoint_jacobian.argtypes = [ctypes.c_int, dp, ctypes.POINTER(OrcOp), ctypes.c_int64, dp,
                                           ctypes.c_int64, dp, ctypes.c_int, i32p, dp, ctypes.c_char_p, dp]
        _lib = L
    return _lib


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def num_threads() -> int:
    return int(lib().orc_num_threads())


def gate_matrix(name: str, angles=(), inverse=False, k=None) -> np.ndarray:
    g = GATES[name]
    if k is None:
        k = {"MultiRZ": 1}.get(name, None) or _own_wires(name)
    dim = 1 << k
    out = np.zeros(dim * dim, dtype=np.complex128)
    ang = np.zeros(3)
    ang[: len(angles)] = angles
    if lib().orc_gate_matrix(g, k, _dptr(ang), int(bool(inverse)), _dptr(out)) != 0:
        raise ValueError(name)
    return out.reshape(dim, dim)


def gate_generator(name: str, k=None):
    g = GATES[name]
    if k is None:
        k = _own_wires(name)
    dim = 1 << k
    out = np.zeros(dim * dim, dtype=np.complex128)
    c = np.zeros(1)
    if lib().orc_gate_generator(g, k, _dptr(out), _dptr(c)) != 0:
        raise ValueError(name)
    return out.reshape(dim, dim), float(c[0])


def _own_wires(name):
    w = lib().orc_gate_wires(GATES[name])
    if w == 0:
        raise ValueError(f"{name} needs an explicit width")
    return w


def _marshal(ops):
    arr = (OrcOp * max(1, len(ops)))()
    mats = []
    moff = 0
    for i, op in enumerate(ops):
        o = arr[i]
        o.gate = GATES[op.name]
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
    matrices = np.concatenate(mats) if mats else np.zeros(1, dtype=np.complex128)
    return arr, matrices


def zero_state(n: int, basis: int = 0) -> np.ndarray:
    psi = np.zeros(1 << n, dtype=np.complex128)
    psi[basis] = 1.0
    return psi


def apply(n: int, ops, params, psi=None) -> np.ndarray:
    """Apply ops to psi (default |0..0>) and return the new state."""
    psi = zero_state(n) if psi is None else np.array(psi, dtype=np.complex128, copy=True)
    params = np.ascontiguousarray(params, dtype=np.float64).reshape(-1)
    if params.size == 0:
        params = np.zeros(1)
    arr, mats = _marshal(ops)
    if lib().orc_apply(n, _dptr(psi), arr, len(ops), _dptr(params), _dptr(mats)) != 0:
        raise ValueError("oracle rejected an operation")
    return psi


def apply_matrix(psi: np.ndarray, wires, mat) -> np.ndarray:
    n = int(np.log2(psi.size))
    out = np.array(psi, dtype=np.complex128, copy=True)
    w = np.ascontiguousarray(wires, dtype=np.int32)
    m = np.ascontiguousarray(mat, dtype=np.complex128)
    lib().orc_apply_matrix(n, _dptr(out), len(w), w.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _dptr(m))
    return out


def inner(a: np.ndarray, b: np.ndarray) -> complex:
    n = int(np.log2(a.size))
    out = np.zeros(2)
    a = np.ascontiguousarray(a, dtype=np.complex128)
    b = np.ascontiguousarray(b, dtype=np.complex128)
    lib().orc_inner(n, _dptr(a), _dptr(b), _dptr(out))
    return complex(out[0], out[1])


def _obs_arrays(observables, n):
    nterms = np.array([len(o.coeffs) for o in observables], dtype=np.int32)
    coeff = np.concatenate([np.asarray(o.coeffs, dtype=np.float64) for o in observables]) if len(observables) else np.zeros(0)
    words = "".join(w for o in observables for w in o.words)
    assert len(words) == n * int(nterms.sum())
    return nterms, np.ascontiguousarray(coeff), words.encode("ascii")


def expval(psi: np.ndarray, observables) -> np.ndarray:
    n = int(np.log2(psi.size))
    psi = np.ascontiguousarray(psi, dtype=np.complex128)
    nterms, coeff, words = _obs_arrays(observables, n)
    out = np.zeros(len(observables))
    if lib().orc_expval(n, _dptr(psi), len(observables), nterms.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                        _dptr(coeff), words, _dptr(out)) != 0:
        raise ValueError("bad Pauli word")
    return out


def apply_pauli_sum(psi: np.ndarray, observable) -> np.ndarray:
    n = int(np.log2(psi.size))
    psi = np.ascontiguousarray(psi, dtype=np.complex128)
    nterms, coeff, words = _obs_arrays([observable], n)
    lam = np.zeros_like(psi)
    if lib().orc_apply_pauli_sum(n, _dptr(psi), int(nterms[0]), _dptr(coeff), words, _dptr(lam)) != 0:
        raise ValueError("bad Pauli word")
    return lam


def adjoint_jacobian(psi: np.ndarray, ops, params, observables) -> np.ndarray:
    """d<O_o>/d params[p] by the adjoint method, from the post-circuit state."""
    n = int(np.log2(psi.size))
    psi = np.ascontiguousarray(psi, dtype=np.complex128)
    params = np.ascontiguousarray(params, dtype=np.float64).reshape(-1)
    n_params = params.size
    if n_params == 0:
        params = np.zeros(1)
    arr, mats = _marshal(ops)
    nterms, coeff, words = _obs_arrays(observables, n)
    jac = np.zeros((len(observables), max(1, n_params)))
    if lib().orc_adjoint_jacobian(n, _dptr(psi), arr, len(ops), _dptr(params), n_params, _dptr(mats),
                                  len(observables), nterms.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                  _dptr(coeff), words, _dptr(jac)) != 0:
        raise ValueError("oracle rejected an operation")
    return jac[:, :n_params]


def sample(psi: np.ndarray, u) -> np.ndarray:
    """Inverse-transform shot sampling with caller-supplied uniforms u in [0, 1)."""
    n = int(np.log2(psi.size))
    psi = np.ascontiguousarray(psi, dtype=np.complex128)
    u = np.ascontiguousarray(u, dtype=np.float64).reshape(-1)
    out = np.zeros(max(1, u.size), dtype=np.int64)
    if lib().orc_sample(n, _dptr(psi), u.size, _dptr(u if u.size else np.zeros(1)),
                        out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))) != 0:
        raise ValueError("zero state")
    return out[:u.size]
