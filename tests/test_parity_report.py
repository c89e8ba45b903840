"""Host-only check of the parity-error report."""
from tests import parity_report


def test_report_groups_and_ratios():
    recs = [{"case": "tests/test_gpu_parity.py::test_a[1-2]", "quantity": "state n=3 seed=1", "dtype": "c64",
             "err": 2e-6, "tol": 1e-5},
            {"case": "tests/test_gpu_parity.py::test_a[3-4]", "quantity": "state n=5 seed=2", "dtype": "c64",
             "err": 4e-6, "tol": 1e-5},
            {"case": "tests/test_gpu_parity.py::test_a[1-2]", "quantity": "jacobian", "dtype": "c128",
             "err": 1e-14, "tol": 1e-12}]
    text = parity_report.report(recs, "cmd")
    assert "| test_gpu_parity.py::test_a | c64 | state | 2 | 4.00e-06 | 1e-05 | 0.400 |" in text
    assert "| test_gpu_parity.py::test_a | c128 | jacobian | 1 | 1.00e-14 | 1e-12 | 0.010 |" in text
    assert "c128: 0.010, c64: 0.400" in text
