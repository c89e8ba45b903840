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
