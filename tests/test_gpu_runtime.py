"""The library and torch share one HIP runtime whatever is used first: a
fresh process that calls into the library (host-only call) before torch has
touched the device must still be able to use torch's device and run an LT
step.  (torch's wheel carries its own HIP runtime; the binding loads torch
before the library so the library's HIP calls bind to it.)"""
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = r"""
import paper_2605_17222_amd as H
import workload as W
H.ckks_lt_autotune(16, 24, 9, H.CKKS_LT_TH_BSGS, 64)   # loads the library first
prm = W.params_toy()
P = H.ckks_params_create(prm.log_n, prm.q, prm.p, prm.dnum)
import torch
x = torch.ones(4, device="cuda")
a = torch.zeros((3, prm.n), dtype=torch.int64, device="cuda")
out = H.empty((3, prm.n))
H.ckks_op_ntt(P, True, 1, 3, a, out)
torch.cuda.synchronize()
assert int(x.sum().item()) == 4 and not out.any().item()
print("ok")
"""


def test_library_first_then_torch():
    env = dict(os.environ, PYTHONPATH=ROOT + os.pathsep + os.environ.get("PYTHONPATH", ""))
    r = subprocess.run([sys.executable, "-c", SCRIPT], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=240)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-2000:]
    assert "ok" in r.stdout
