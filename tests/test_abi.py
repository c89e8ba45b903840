"""C-ABI boundary checks that need no GPU: the library loads, exports every
symbol include/qsv.h declares, and host-side validation rejects bad input
before any device work."""
import os
import re

import numpy as np
import pytest

from paper_2403_02512_amd import qsv
from paper_2403_02512_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "qsv.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(qsv_[a-z_]+)\s*\(", src)))


def test_header_declares_the_binding_exports():
    assert declared_functions() == sorted(qsv.EXPORTS)


def test_library_exports_every_declared_symbol():
    import ctypes
    L = ctypes.CDLL(qsv.LIB_PATH)
    for name in declared_functions():
        assert hasattr(L, name), name
    assert qsv.lib().qsv_version().decode().startswith("qsv")


def test_device_count_without_gpu_is_not_an_error():
    assert qsv.device_count() >= 0


def test_status_strings():
    L = qsv.lib()
    for st, s in qsv.STATUS.items():
        assert L.qsv_status_string(st).decode() == s


def _err(fn):
    with pytest.raises(qsv.QsvError) as e:
        fn()
    return e.value.status


def test_validation_errors():
    ok = [W.op("RX", [0], (0, 1.0)), W.op("CNOT", [0, 2])]
    qsv.validate_ops(3, ok, 1)
    assert _err(lambda: qsv.validate_ops(3, [W.op("RX", [3], (0, 1.0))], 1)) == -2        # wire range
    assert _err(lambda: qsv.validate_ops(3, [W.op("CNOT", [1, 1])], 0)) == -2             # repeated wire
    assert _err(lambda: qsv.validate_ops(3, [W.op("CNOT", [1])], 0)) == -2                # wire count
    assert _err(lambda: qsv.validate_ops(3, [W.op("RX", [0], (5, 1.0))], 1)) == -7        # param index
    assert _err(lambda: qsv.validate_ops(0, ok, 1)) == -1                                 # n_qubits
    assert _err(lambda: qsv.validate_ops(35, ok, 1)) == -1
    bad_ctrl = W.op("RX", [0, 1], (0, 1.0), n_ctrls=1, ctrl_values=2)
    assert _err(lambda: qsv.validate_ops(3, [bad_ctrl], 1)) == -1                         # ctrl value bits
    wide = W.op("QubitUnitary", list(range(7)), matrix=np.eye(128))
    assert _err(lambda: qsv.validate_ops(8, [wide], 0)) == -6                             # > 6 targets
    # matrix offset beyond the matrices array
    m = qsv.MarshalledOps([W.op("QubitUnitary", [0], matrix=np.eye(2))], np.zeros(0))
    m.arr[0].matrix_offset = 3
    st = qsv.lib().qsv_validate_ops(2, m.arr, 1, 0, m.n_mat)
    assert st == -7


def test_every_gate_validates():
    for name, (k, na) in W.GATE_ARITY.items():
        k = k or 2
        mat = np.eye(1 << k) if name == "QubitUnitary" else None
        qsv.validate_ops(4, [W.op(name, list(range(k)), *[(0, 1.0)] * na, matrix=mat)], 1)


def test_observable_validation():
    qsv.validate_obs(3, [W.PauliSum(np.array([1.0, 2.0]), ["XYZ", "IIZ"])])
    with pytest.raises(ValueError):
        qsv.validate_obs(3, [W.PauliSum(np.array([1.0]), ["XQZ"])])
    m = qsv.MarshalledObs([W.PauliSum(np.array([1.0]), ["ZZZZ"])])
    assert qsv.lib().qsv_validate_obs(3, m.arr, 1) == -2                                   # mask beyond n


def test_context_creation_fails_cleanly_without_device():
    if qsv.device_count() > 0:
        pytest.skip("a GPU is present")
    assert _err(lambda: qsv.Context(0)) == -1
    assert "no HIP device" in qsv.lib().qsv_thread_last_error().decode()


def test_pauli_mask_convention():
    # wire 0 is the most significant index bit; Y sets both masks
    assert qsv.pauli_masks("XIZ") == (0b100, 0b001)
    assert qsv.pauli_masks("IYI") == (0b010, 0b010)
