"""The C++ example (csrc/pmace_demo.cpp) drives the C ABI with no Python in
the process: device simulation of the measurements (eq. (1), eq. (16)), PMACE
iterations (Alg. 1) and the data-fit cost of eq. (4).  Checked here: it exits
cleanly, the cost falls, and the reconstruction approaches the object."""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
DEMO = os.path.join(os.path.dirname(HERE), "paper_2111_14240_amd", "pmace_demo")


def _run(args):
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    if not os.path.exists(DEMO):
        pytest.fail("pmace_demo is not built (paper_2111_14240_amd/build.py)")
    print("[gpu-demo]", " ".join(map(str, args)), flush=True)
    sys.stdout.flush()
    res = subprocess.run([DEMO, *map(str, args)], capture_output=True, text=True, timeout=120)
    print(res.stdout, res.stderr, flush=True)
    assert res.returncode == 0, res.stderr
    lines = res.stdout.strip().splitlines()
    costs = [float(l.split()[-1]) for l in lines if l.startswith("iteration")]
    return costs, json.loads(lines[-1])


@pytest.mark.parametrize("args", [(256, 64, 8, 24, 1e5, 60), (512, 128, 15, 24, 1e5, 100),
                                  (640, 192, 10, 48, 1e6, 40)])
def test_demo(args):
    costs, out = _run(args)
    assert out["iterations"] == args[-1] and out["positions"] == args[2] ** 2
    assert costs[-1] < 0.2 * costs[0], costs
    assert out["nrmse"] < 0.3, out
