"""Patches per workgroup of the whole-patch agent (pmace_params.ppw).

Each patch of a workgroup runs the same steps on its own LDS tile, so every
choice gives bitwise the same iteration as one patch per workgroup, including
the partly filled last workgroup (J not a multiple of ppw) and, in a batch,
workgroups whose patches belong to members that stop at different
iterations.  One pass is also checked against the FP64 oracle directly."""
import sys

import numpy as np
import pytest

from oracle import pmace_oracle as O
from paper_2111_14240_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

MAX_PPW = {32: 8, 48: 4, 64: 2}


def _say(*a):
    print("[gpu-ppw]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2111_14240_amd import pmace
    pmace.load_library()
    return pmace


def _run(P, prob, ppw, iters, **kw):
    R = P.Reconstruction(prob.n1, prob.n2, prob.probe, prob.pos, prob.z, 0.5, ppw=ppw, **kw)
    R.iterate(iters)
    out = R.get_state().cpu().numpy(), R.reconstruct().cpu().numpy()
    R.close()
    return out


@pytest.mark.parametrize("np_,n,scan,step", [(32, 160, 5, 30), (48, 200, 5, 36), (64, 256, 5, 44)])
def test_ppw_bitwise_equal_to_one_patch_per_workgroup(P, np_, n, scan, step):
    prob = synth.make_problem(n, np_, scan, step, 1e5, 60 + np_)
    assert len(prob.pos) % 2 == 1          # a partly filled last workgroup for every ppw > 1
    v1, x1 = _run(P, prob, 1, 4)
    k = 2
    while k <= MAX_PPW[np_]:
        _say("np", np_, "J", len(prob.pos), "ppw", k)
        v, x = _run(P, prob, k, 4)
        assert np.array_equal(v, v1) and np.array_equal(x, x1), k
        k *= 2


def test_ppw_sharp_plus_bitwise(P):
    prob = synth.make_problem(160, 32, 5, 30, 1e5, 70)
    kw = dict(method=P.PMACE_METHOD_SHARP_PLUS, beta=0.8)
    v1, x1 = _run(P, prob, 1, 3, **kw)
    v8, x8 = _run(P, prob, 8, 3, **kw)
    assert np.array_equal(v1, v8) and np.array_equal(x1, x8)


def test_ppw_pass_matches_oracle(P):
    """One teacher-forced pass with 4 patches per workgroup, from a smooth start,
    against the oracle at 1e-4 (L2 and element-wise)."""
    prob = synth.make_problem(200, 48, 5, 36, 1e5, 71)
    d = prob.probe.astype(np.complex64).astype(np.complex128)
    y = O.amplitudes(prob.z.astype(np.float32))
    shape = (prob.n1, prob.n2)
    v0 = O.extract(synth.make_object(prob.n1, prob.n2, np.random.default_rng(5)), prob.pos, prob.np_)
    v1, _, _ = O.pmace_step(v0, d, y, prob.pos, shape, 0.5, 1.25, 0.5)
    R = P.Reconstruction(prob.n1, prob.n2, prob.probe, prob.pos, prob.z, 0.5, ppw=4)
    R.set_state(v0)
    R.iterate(1)
    v = R.get_state().cpu().numpy().astype(np.complex128)
    R.close()
    e = np.linalg.norm(v - v1) / np.linalg.norm(v1)
    m = np.max(np.abs(v - v1)) / np.max(np.abs(v1))
    _say("ppw 4 pass vs oracle", e, m)
    assert e < 1e-4 and m < 1e-4


def test_batch_ppw_with_members_stopping_apart(P):
    """A batch whose Np = 32 class runs 8 patches per workgroup (its first
    member's choice): member A, 3 iterations ahead, stops 3 iterations before
    B and C while sharing workgroups with B; every member must equal the same
    reconstruction advanced alone for its number of iterations."""
    probs = [synth.make_problem(96, 32, 2, 24, 1e5, 72),    # J = 4
             synth.make_problem(112, 32, 3, 24, 1e5, 73),   # J = 9
             synth.make_problem(128, 32, 5, 20, 1e5, 74)]   # J = 25
    K = 6
    Rs = [P.Reconstruction(p.n1, p.n2, p.probe, p.pos, p.z, 0.5, ppw=8 if i == 0 else 1)
          for i, p in enumerate(probs)]
    B0 = P.Batch([Rs[0]], tol=0.0, min_iter=0, max_iter=100)
    B0.step(3)
    B0.close()
    B = P.Batch(Rs, tol=0.0, min_iter=0, max_iter=K)
    B.step(K + 2)
    done, _, iters = B.poll()
    _say("iterations", iters.tolist())
    assert done.tolist() == [1, 1, 1] and iters.tolist() == [K, K, K]
    for i, (R, p) in enumerate(zip(Rs, probs)):
        v, x = _run(P, p, 1, K)
        assert np.array_equal(R.get_state().cpu().numpy(), v), i
        assert np.array_equal(R.reconstruct().cpu().numpy(), x), i
    B.close()
    for R in Rs:
        R.close()
