"""The library and PyTorch share one HIP runtime whatever is imported first
(regression: with the library loaded before torch, torch found no GPU)."""
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = """
import numpy as np
from paper_2403_02512_amd import qsv
ctx = qsv.Context(0)
st = qsv.State(ctx, 4)
st.reset(3)
assert abs(st.to_numpy()[3] - 1) == 0
import torch
t = torch.zeros(16, dtype=torch.complex128, device="cuda")
st2 = qsv.State(ctx, 4, tensor=t)
st2.reset(5)
torch.cuda.synchronize()
assert t[5].item() == 1
print("ok")
"""


def test_library_before_torch_in_a_fresh_process():
    r = subprocess.run([sys.executable, "-c", SCRIPT], cwd=ROOT, capture_output=True, text=True, timeout=240)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), r.stdout + r.stderr
