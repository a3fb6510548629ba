"""A system created before any PyTorch call leaves PyTorch's GPU usable (the
binding initialises PyTorch's HIP runtime before loading the library's).
Runs in a fresh interpreter, since this test process has initialised the GPU
already.  Needs an MI355X.
"""
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = """
import sys
sys.path.insert(0, {root!r})
from paper_2311_11322_amd import dem, workloads as W
w = W.periodic_box(5, n_agg=50)
s = dem.Sim(w.params)
s.add_workload(w)
s.step(2)
import torch
x = torch.arange(8, dtype=torch.float64, device="cuda")
torch.cuda.synchronize()
assert float(x.sum().item()) == 28.0
print("ok", s.read_state(["agg_pos"])["agg_pos"].shape)
"""


def test_system_before_torch_leaves_torch_usable():
    print("[case] system before torch, fresh interpreter", flush=True)
    r = subprocess.run([sys.executable, "-c", SCRIPT.format(root=ROOT)], capture_output=True,
                       text=True, timeout=240)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-2000:]
    assert "ok" in r.stdout
