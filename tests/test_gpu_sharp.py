"""SHARP+ (Alg. 2) on the device against the FP64 oracle.

The device carries one overlap projection per iteration (P_Q s_{k+1} =
P_Q P_a s_k); the oracle applies Alg. 2 as written, with two.  Bar: relative
error <= 1e-4 per teacher-forced iteration on the frames s and on the output."""
import sys

import numpy as np
import pytest

from oracle import pmace_oracle as O
from paper_2111_14240_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
TOL = 1e-4

STAGED, ROWSPEC = 0x2, 0x8   # PMACE_STAGED_AGENT, PMACE_ROWSPEC_AGENT

CASES = {
    # name: (n, np, scan, step, peak, seed, chunk, agent flags)
    "np32": (128, 32, 6, 16, None, 1, 0, 0),
    "np64": (200, 64, 5, 30, 1e5, 21, 0, 0),
    "np128": (320, 128, 4, 56, 1e5, 22, 0, 0),
    "np256_ragged_chunks": (400, 256, 3, 60, 1e6, 23, 4, STAGED),
    "np96": (288, 96, 5, 40, 1e5, 52, 0, 0),
    "np192_chunks": (400, 192, 3, 90, 1e5, 54, 4, STAGED),
    # the states kept as row spectra (SHARP+ has no zero rule, so any probe)
    "np256_rowspec_chunks": (400, 256, 3, 60, 1e6, 23, 4, ROWSPEC),
    "np192_rowspec": (400, 192, 3, 90, 1e5, 54, 0, ROWSPEC),
    "np160_rowspec_chunks": (360, 160, 3, 80, 1e6, 53, 4, ROWSPEC),
}


def _say(*a):
    print("[gpu-sharp]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2111_14240_amd import pmace
    pmace.load_library()
    return pmace


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.complex128) - b) / np.linalg.norm(b))


@pytest.mark.parametrize("case", sorted(CASES))
@pytest.mark.parametrize("beta", [0.5, 0.8])
def test_sharp_plus_teacher_forced(P, case, beta):
    n, np_, scan, step, peak, seed, chunk, flags = CASES[case]
    prob = synth.make_problem(n, np_, scan, step, peak, seed)
    d = prob.probe.astype(np.complex64).astype(np.complex128)
    y = O.amplitudes(prob.z)
    shape = (n, n)
    x0 = synth.make_object(n, n, np.random.default_rng(99))
    ss = [O.sharp_plus_init(x0, d, prob.pos)]
    for _ in range(4):
        ss.append(O.sharp_plus_step(ss[-1], d, y, prob.pos, shape, beta))
    _say(case, "beta", beta)
    R = P.Reconstruction(n, n, prob.probe, prob.pos, prob.z, 0.0, x0=x0.astype(np.complex64),
                         chunk=chunk, method=P.PMACE_METHOD_SHARP_PLUS, beta=beta, flags=flags)
    if flags == ROWSPEC:
        assert R.agent == "row-spectrum"
    s0 = R.get_state().cpu().numpy()
    assert rel(s0, ss[0]) < 1e-6
    for k in range(4):
        R.set_state(ss[k])
        assert rel(R.get_state().cpu().numpy(), ss[k]) < 1e-6
        R.iterate(1)
        es = rel(R.get_state().cpu().numpy(), ss[k + 1])
        ex = rel(R.reconstruct().cpu().numpy(), O.sharp_plus_reconstruct(ss[k + 1], d, prob.pos, shape))
        _say(f"  k={k} rel(s)={es:.2e} rel(xhat)={ex:.2e}")
        assert es < TOL and ex < TOL
    # free-running from x0 follows the same trajectory for a few steps
    R2 = P.Reconstruction(n, n, prob.probe, prob.pos, prob.z, 0.0, x0=x0.astype(np.complex64),
                          chunk=chunk, method=P.PMACE_METHOD_SHARP_PLUS, beta=beta, flags=flags)
    R2.iterate(4)
    assert rel(R2.get_state().cpu().numpy(), ss[4]) < 10 * TOL
    R.close()
    R2.close()


def elem(a, b):
    """Element by element: the largest pointwise error over the largest value."""
    a = np.asarray(a, np.complex128)
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


@pytest.mark.slow
@pytest.mark.parametrize("config,flags", [("c3", 0), ("c3", STAGED), ("c3", ROWSPEC), ("c2", 0)])
def test_sharp_plus_full_size(P, config, flags):
    """SHARP+ on the full C3 (1024^2 object, 1600 positions of 256^2; the
    default agent, and the three-pass and row-spectrum agents) and C2 (512^2,
    225 of 128^2) workloads in the launch configuration bench.py --method
    sharp times (beta 0.8, tuned chunks): the first pass from a smooth start
    and a teacher-forced second pass, on every frame."""
    beta = 0.8
    prob = synth.make_config_problem(config)
    n = prob.n1
    d = prob.probe.astype(np.complex64).astype(np.complex128)
    y = O.amplitudes(prob.z.astype(np.float32))
    shape = (n, n)
    x0 = synth.make_object(n, n, np.random.default_rng(99))
    _say(f"{config} sharp+: oracle, 2 steps")
    ss = [O.sharp_plus_init(x0, d, prob.pos)]
    for _ in range(2):
        ss.append(O.sharp_plus_step(ss[-1], d, y, prob.pos, shape, beta))
    R = P.Reconstruction(n, n, prob.probe, prob.pos, prob.z, 0.5, x0=x0.astype(np.complex64),
                         method=P.PMACE_METHOD_SHARP_PLUS, beta=beta, flags=flags)
    _say(f"  agent: {R.agent}")
    for k in range(2):
        if k:
            R.set_state(ss[k])
        R.iterate(1)
        s1 = R.get_state().cpu().numpy()
        xr = O.sharp_plus_reconstruct(ss[k + 1], d, prob.pos, shape)
        xh = R.reconstruct().cpu().numpy()
        es, ex = rel(s1, ss[k + 1]), rel(xh, xr)
        ms, mx = elem(s1, ss[k + 1]), elem(xh, xr)
        _say(f"  k={k} rel(s)={es:.2e} rel(xhat)={ex:.2e} elementwise {ms:.2e} {mx:.2e}")
        assert es < TOL and ex < TOL and ms < TOL and mx < TOL
    R.close()


@pytest.mark.parametrize("case,iters", [("c1", 50), ("np256_ragged_chunks", 20), ("np256_rowspec_chunks", 20)])
def test_sharp_plus_every_iteration(P, case, iters):
    """SHARP+ teacher-forced at every iteration of a longer run from a smooth
    start (beta 0.8): the C1 workload to 50 iterations on the whole-patch agent,
    and a case with ragged chunks to 20 on the three-pass and on the
    row-spectrum agent, each pass on every frame and on the output, in L2 and
    element by element."""
    beta = 0.8
    if case == "c1":
        prob = synth.make_config_problem("c1")
        chunk, flags = 0, 0
    else:
        n, np_, scan, step, peak, seed, chunk, flags = CASES[case]
        prob = synth.make_problem(n, np_, scan, step, peak, seed)
    n = prob.n1
    d = prob.probe.astype(np.complex64).astype(np.complex128)
    y = O.amplitudes(prob.z.astype(np.float32))
    shape = (n, n)
    x0 = synth.make_object(n, n, np.random.default_rng(98))
    _say(case, "sharp+ oracle trajectory", iters)
    ss = [O.sharp_plus_init(x0, d, prob.pos)]
    for _ in range(iters):
        ss.append(O.sharp_plus_step(ss[-1], d, y, prob.pos, shape, beta))
    R = P.Reconstruction(n, n, prob.probe, prob.pos, prob.z, 0.0, x0=x0.astype(np.complex64),
                         chunk=chunk, method=P.PMACE_METHOD_SHARP_PLUS, beta=beta, flags=flags)
    worst = 0.0
    for k in range(iters):
        R.set_state(ss[k])
        R.iterate(1)
        s1 = R.get_state().cpu().numpy()
        xr = O.sharp_plus_reconstruct(ss[k + 1], d, prob.pos, shape)
        xh = R.reconstruct().cpu().numpy()
        errs = (rel(s1, ss[k + 1]), rel(xh, xr), elem(s1, ss[k + 1]), elem(xh, xr))
        if k % 10 == 0 or k == iters - 1:
            _say(f"  k={k} rel(s)={errs[0]:.2e} rel(xhat)={errs[1]:.2e} elementwise {errs[2]:.2e} {errs[3]:.2e}")
        assert max(errs) < TOL, (k, errs)
        worst = max(worst, max(errs))
    _say(f"  worst = {worst:.2e}")
    R.close()


def test_sharp_plus_rowspec_row_segments(P):
    """SHARP+ on row-spectrum states over a 400 x 1280 object whose 3 x 12
    positions of 192^2 cross column 1024 (object rows summed in two
    segments, patches straddling them; consensus over the stage's projected
    frames), chunks of 8 positions: teacher-forced at every iteration to 10
    from a smooth start, beta 0.8, on every frame and on the output."""
    beta = 0.8
    prob = synth.make_problem(400, 192, 3, 96, 1e5, 61, n2=1280, scan2=12)
    assert prob.pos[:, 1].min() < 1024 - 192 and prob.pos[:, 1].max() > 1024
    n1, n2 = prob.n1, prob.n2
    d = prob.probe.astype(np.complex64).astype(np.complex128)
    y = O.amplitudes(prob.z.astype(np.float32))
    shape = (n1, n2)
    x0 = synth.make_object(n1, n2, np.random.default_rng(97))
    ss = [O.sharp_plus_init(x0, d, prob.pos)]
    for _ in range(10):
        ss.append(O.sharp_plus_step(ss[-1], d, y, prob.pos, shape, beta))
    R = P.Reconstruction(n1, n2, prob.probe, prob.pos, prob.z, 0.0, x0=x0.astype(np.complex64), chunk=8,
                         method=P.PMACE_METHOD_SHARP_PLUS, beta=beta, flags=ROWSPEC)
    assert R.agent == "row-spectrum"
    worst = 0.0
    for k in range(10):
        R.set_state(ss[k])
        R.iterate(1)
        s1 = R.get_state().cpu().numpy()
        xr = O.sharp_plus_reconstruct(ss[k + 1], d, prob.pos, shape)
        xh = R.reconstruct().cpu().numpy()
        errs = (rel(s1, ss[k + 1]), rel(xh, xr), elem(s1, ss[k + 1]), elem(xh, xr))
        assert max(errs) < TOL, (k, errs)
        worst = max(worst, max(errs))
    _say(f"  row segments, sharp+ worst = {worst:.2e}")
    R.close()
