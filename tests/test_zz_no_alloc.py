"""The allocation-free simulate entry point against pmace_simulate (the same
kernels on a caller's workspace): equal bit for bit on two calls in a row,
the second smaller, plus its size limit and its device-side position check."""
import ctypes
import sys

import numpy as np
import pytest

from paper_2111_14240_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu-noalloc]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2111_14240_amd import pmace
    pmace.load_library()
    return pmace


def _inputs(n, np_, scan, step, seed):
    prob = synth.make_problem(n, np_, scan, step, None, seed=seed)
    return prob.x_true, prob.probe, prob.pos


@pytest.mark.parametrize("peak", [None, 1e5])
def test_static_equals_workspace_two_calls(P, peak):
    # first call: Np = 256 with 100 positions (51 MiB of frames in the scratch),
    # second: a smaller Np = 160 problem, then a fused-side one (Np = 64)
    for (n, np_, scan, step, seed) in [(512, 256, 10, 28, 5), (320, 160, 5, 40, 6), (200, 64, 6, 27, 7)]:
        x, d, pos = _inputs(n, np_, scan, step, seed)
        _say("case", n, np_, len(pos), peak)
        assert len(pos) * np_ * np_ * 8 <= P.simulate_static_max_bytes()
        z_ws, s_ws = P.simulate(x, d, pos, peak, seed=11)
        z_st, s_st = P.simulate_static(x, d, pos, peak, seed=11)
        torch.cuda.synchronize()
        assert s_ws == s_st
        a, b = z_ws.cpu().numpy(), z_st.cpu().numpy()
        assert np.array_equal(a.view(np.uint32), b.view(np.uint32)), np.abs(a - b).max()


def test_static_limit_and_bad_position(P):
    x, d, pos = _inputs(512, 256, 12, 21, 8)
    assert len(pos) * 256 * 256 * 8 > P.simulate_static_max_bytes()
    with pytest.raises(RuntimeError, match="pmace_simulate_static"):
        P.simulate_static(x, d, pos, None, seed=1)
    x, d, pos = _inputs(200, 64, 4, 40, 9)
    pos = np.array(pos, dtype=np.int32)
    pos[2, 1] = 200 - 64 + 1   # leaves the object by one column
    with pytest.raises(RuntimeError, match="pmace_simulate_static"):
        P.simulate_static(x, d, pos, None, seed=1)
    # the array is usable again afterwards
    pos[2, 1] = 0
    z_ws, _ = P.simulate(x, d, pos, 1e4, seed=3)
    z_st, _ = P.simulate_static(x, d, pos, 1e4, seed=3)
    assert np.array_equal(z_ws.cpu().numpy(), z_st.cpu().numpy())
