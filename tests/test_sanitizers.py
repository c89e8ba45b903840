"""The library's host runtime (validation, planning, lowering, C entry
points) and the CPU oracle, built with AddressSanitizer and
UndefinedBehaviorSanitizer and run on a host workload in a child process
(tests/sanitized_workload.py).  Any sanitizer report aborts the child."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
OUT = os.path.join(ROOT, "_build", "sanitize")
WORKLOAD = os.path.join(ROOT, "tests", "sanitized_workload.py")


def _run(which, env):
    e = dict(os.environ)
    e.update(env)
    e["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"       # the interpreter's own leaks are not ours
    e["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    r = subprocess.run([sys.executable, WORKLOAD, which], env=e, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, f"{which} under sanitizers failed:\n{r.stdout[-3000:]}\n{r.stderr[-6000:]}"
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error:" not in r.stderr, r.stderr[-6000:]
    return r.stdout


@pytest.mark.skipif(shutil.which("hipcc") is None and not os.path.exists("/opt/rocm/bin/hipcc"),
                    reason="hipcc is needed to build the library")
def test_host_runtime_under_asan_ubsan():
    from paper_2403_02512_amd import build
    lib = build.build_sanitized(OUT)
    rt = build.asan_runtime()
    assert os.path.exists(rt), rt
    out = _run("qsv", {"QSV_LIB_PATH": lib, "LD_PRELOAD": rt})
    assert "qsv host runtime: ok" in out


def test_oracle_under_asan_ubsan():
    import oracle.oracle as orc
    lib = orc.build_sanitized(OUT)
    rt = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    out = _run("oracle", {"ORACLE_LIB_PATH": lib, "LD_PRELOAD": rt})
    assert "oracle: ok" in out
