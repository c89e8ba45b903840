"""Record of the errors the GPU parity tests measure against the oracle.

Every check that goes through tests/gpu_helpers.py adds one record (case,
quantity, precision, error, tolerance).  When the environment variable
QSV_PARITY_LOG names a file, the session appends its records there as JSON
lines; tests/parity_report.py turns them into the committed table of
achieved errors.  No product code is imported here.
"""
import json
import os

RECORDS = []


def record(case: str, quantity: str, dtype: str, err: float, tol: float, **extra) -> None:
    RECORDS.append({"case": case, "quantity": quantity, "dtype": dtype, "err": float(err), "tol": float(tol),
                    **extra})


def flush() -> None:
    path = os.environ.get("QSV_PARITY_LOG")
    if not path or not RECORDS:
        return
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    with open(path, "a") as f:
        for r in RECORDS:
            f.write(json.dumps(r) + "\n")
    RECORDS.clear()
