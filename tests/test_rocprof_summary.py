"""Host-only checks of the rocprofv3 summariser used for profiles/."""
import csv
import os

from paper_2403_02512_amd import rocprof_summary as rs


def _write_counters(path, counter, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for name, val in rows:
            w.writerow({"Kernel_Name": name, "Counter_Name": counter, "Counter_Value": val})


def test_traffic_calibration_and_source_check(tmp_path):
    B = 4294967296.0
    fetch = tmp_path / "f.csv"
    write = tmp_path / "w.csv"
    # the copy reads half its bytes on the counter, writes them all
    _write_counters(fetch, "FETCH_SIZE", [("__amd_rocclr_copyBuffer", B / 2 / 1024), ("__amd_rocclr_copyBuffer", 0),
                                          ("void qsv::k_tile<double, true, 3, false>(...)", B / 1024),
                                          ("void qsv::k_tile<double, true, 3, false>(...)", B / 1024)])
    _write_counters(write, "WRITE_SIZE", [("__amd_rocclr_copyBuffer", B / 1024), ("__amd_rocclr_copyBuffer", 0),
                                          ("void qsv::k_tile<double, true, 3, false>(...)", 2 * B / 1024),
                                          ("void qsv::k_tile<double, true, 3, false>(...)", 2 * B / 1024)])
    text = rs.traffic(str(fetch), str(write), B, "cmd")
    assert "fetch_scale=2.0000 write_scale=1.0000" in text
    out = tmp_path / "t.txt"
    out.write_text(text)
    kv = rs.read_traffic(str(out))
    # 2 B fetched (scaled) + 2 B written per launch; the summary keeps 5 digits
    assert set(kv) == {"tile2"} and abs(kv["tile2"] - 4 * B) <= 1e-4 * 4 * B
    # a summary taken on another kernel source is not used
    out.write_text(text.replace(rs.source_sha1(), "0" * 40))
    assert rs.read_traffic(str(out)) is None
    assert rs.read_traffic(str(tmp_path / "missing.txt")) is None


def test_kernel_kinds():
    assert rs.kind_of("void qsv::k_tile<double, false, 4, false>(x)") == "tile1"
    assert rs.kind_of("void qsv::k_pauli<float, true, false>(x)") == "other"
    assert rs.kind_of("void qsv::k_pauli<double, true, false>(x)") == "pauli_lambda"
    assert rs.kind_of("__amd_rocclr_copyBuffer") == "copy"


def test_source_hash_covers_every_library_source(tmp_path):
    # the counters are retired by a change to any source under csrc/, not
    # only the kernels: the planner and lowering decide the launched programs
    for name in ("kernels.hip", "plan.cpp", "api.cpp"):
        (tmp_path / name).write_text("x")
    h0 = rs.source_sha1(str(tmp_path))
    (tmp_path / "plan.cpp").write_text("y")
    h1 = rs.source_sha1(str(tmp_path))
    (tmp_path / "new.h").write_text("")
    h2 = rs.source_sha1(str(tmp_path))
    assert len({h0, h1, h2}) == 3
    assert rs.source_sha1() == rs.source_sha1(rs.CSRC)


def test_sweep_traffic_splits_cases_at_markers(tmp_path):
    import json
    n, reps = 10, 2
    state = float(1 << n) * 16
    fill = "void at::native::vectorized_elementwise_kernel<4, at::native::FillFunctor<float> >(...)"
    gate = "void qsv::k_diag1<double>(...)"
    # dispatch order: a fill (the marker tensor's creation), a launch, the copy (calibration: the
    # fetch counter reads half), then per case
    # a warm-up launch, the marker and `reps` timed launches
    seq = [(fill, 0.0, 256.0), (gate, 1.0, 1.0), ("__amd_rocclr_copyBuffer", state / 2, state)]
    per_case = [(0.5 * state, 0.5 * state), (2 * state, 2 * state)]
    for f, w in per_case:
        seq.append((gate, 7.0, 7.0))
        seq.append((fill, 0.0, 256.0))
        seq += [(gate, f / 2, w)] * reps
    for counter, col, path in (("FETCH_SIZE", 1, tmp_path / "f.csv"), ("WRITE_SIZE", 2, tmp_path / "w.csv")):
        with open(path, "w", newline="") as fh:
            wr = csv.DictWriter(fh, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
            wr.writeheader()
            for i, row in enumerate(seq):
                wr.writerow({"Dispatch_Id": i + 1, "Kernel_Name": row[0], "Counter_Name": counter,
                             "Counter_Value": row[col] / 1024})
    log = tmp_path / "s.log"
    log.write_text("\n".join(json.dumps({"case": f"c{i}", "n_qubits": n, "dtype": "c128", "alg_GB": state / 1e9,
                                         "ms": 1.0, "kernels": {"diag1": 1}}) for i in range(2)) + "\n")
    text = rs.sweep_traffic(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), str(log), reps, "cmd")
    assert "fetch_scale=2.0000 write_scale=1.0000" in text
    rows = [l for l in text.splitlines() if l.startswith("| c") and not l.startswith("| case")]
    # case 0 moves its algorithmic bytes, case 1 four times them; warm-up launches are not counted
    assert "| 1.00 |" in rows[0] and "| 4.00 |" in rows[1]
