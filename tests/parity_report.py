"""Turn the parity-error records of a GPU test session (QSV_PARITY_LOG, JSON
lines written by tests/parity_log.py) into the committed markdown table of
achieved errors against the oracle.

  python -m tests.parity_report <records.jsonl> --cmd "<command>" > tests/results/parity_errors_gpu.md

One row per (test, precision, quantity): the number of checks, the largest
error, the tolerance asserted, and the largest error / tolerance ratio.
"""
import argparse
import collections
import json
import re
import sys


def _test_of(case: str) -> str:
    # "tests/test_gpu_parity.py::test_x[...] (call)" -> "test_gpu_parity.py::test_x"
    base = case.split("[")[0]
    return base.split("/")[-1]


def _quantity(q: str) -> str:
    # drop per-case detail (wires, seeds, circuit ids) from the quantity name
    q = re.sub(r" n=.*$", "", q)
    q = re.sub(r" circuit \d+ \(.*\)$", "", q)
    q = re.sub(r" \[.*\]$", "", q)
    return q.strip() or "state"


def report(records, cmd: str) -> str:
    rows = collections.OrderedDict()
    for r in records:
        key = (_test_of(r["case"]), r["dtype"], _quantity(r["quantity"]))
        d = rows.setdefault(key, {"n": 0, "err": 0.0, "tol": r["tol"], "ratio": 0.0})
        d["n"] += 1
        d["err"] = max(d["err"], r["err"])
        d["tol"] = max(d["tol"], r["tol"])
        d["ratio"] = max(d["ratio"], r["err"] / r["tol"] if r["tol"] > 0 else float("inf"))
    out = [f"command: {cmd}", "",
           "Achieved errors of the HIP path against the FP64 oracle (or, where marked, a closed form or the GPU's "
           "own shift rule), per test, precision and quantity. Errors are the readings of the tolerance: state "
           "vectors by ||psi - psi_ref||_2, expectation values relative to sum |c_t|, Jacobian entries relative to "
           "their bound.", "",
           "| test | dtype | quantity | checks | max error | tolerance | max error / tolerance |",
           "|---|---|---|---|---|---|---|"]
    esc = lambda x: x.replace("|", "\\|")  # a literal bar inside a table cell
    for (t, dt, q), d in sorted(rows.items(), key=lambda kv: (kv[0][1], kv[0][0], kv[0][2])):
        out.append(f"| {esc(t)} | {dt} | {esc(q)} | {d['n']} | {d['err']:.2e} | {d['tol']:.0e} | {d['ratio']:.3f} |")
    worst = {}
    for (t, dt, q), d in rows.items():
        worst[dt] = max(worst.get(dt, 0.0), d["ratio"])
    out += ["", "Largest error / tolerance per precision: " +
            ", ".join(f"{dt}: {v:.3f}" for dt, v in sorted(worst.items())),
            f"Checks recorded: {sum(d['n'] for d in rows.values())}"]
    return "\n".join(out) + "\n"


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("records")
    ap.add_argument("--cmd", required=True)
    a = ap.parse_args(argv)
    recs = [json.loads(l) for l in open(a.records) if l.strip()]
    sys.stdout.write(report(recs, a.cmd))


if __name__ == "__main__":
    main()
