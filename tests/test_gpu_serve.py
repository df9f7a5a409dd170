"""The continuous-batching server on the device: requests admitted and retired
while others run (batches rebuilt on every change, large requests optionally
in a batch and stream of their own) end with exactly the reconstruction and
iteration count of the same request solved alone."""
import sys

import numpy as np
import pytest

from paper_2111_14240_amd import serve, synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

MIX = [  # (n, np, scan, step, peak, seed): patch pixels per iteration 37K .. 262K
    (128, 32, 6, 16, 1e5, 71),
    (200, 64, 5, 30, 1e5, 72),
    (300, 256, 2, 40, 1e5, 73),
    (320, 128, 4, 56, 1e5, 74),
    (160, 64, 4, 28, 1e5, 75),
    (400, 192, 2, 100, 1e5, 76),
]
RULE = dict(tol=1e-4, min_iter=2, max_iter=60)


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2111_14240_amd import pmace
    pmace.load_library()
    return pmace


def _tick(clock, n_active, iters):
    clock.advance(1e-3 * iters)


@pytest.mark.parametrize("split", [None, 200000])
def test_served_equals_alone(P, split):
    probs = [synth.make_problem(*m) for m in MIX]

    def requests():
        return [serve.Request(i, p, 0.002 * i) for i, p in enumerate(probs)]

    print("[gpu-serve] split", split, flush=True)
    sys.stdout.flush()
    served = requests()
    ex = serve.GPUExecutor(alpha=0.5, split_work=split, **RULE)
    st = serve.Server(ex, 1 << 40, iters_per_step=3, on_step=_tick, large_work=split).run(
        served, serve.FakeClock())
    assert st.completed == len(MIX) and st.max_active > 1
    alone = requests()
    serve.run_plain(serve.GPUExecutor(alpha=0.5, **RULE), alone, serve.FakeClock(), iters_per_step=3,
                    on_step=_tick)
    for a, b in zip(served, alone):
        print(f"  request {a.rid}: {a.iters} iterations served, {b.iters} alone", flush=True)
        assert a.iters == b.iters and a.nrmse == b.nrmse
        assert np.array_equal(a.result, b.result)


def test_served_request_matches_oracle(P):
    """One request served beside others (admitted while they run), from a
    smooth start, for a fixed number of iterations: its reconstruction equals
    the FP64 oracle's at 1e-4, in L2 and element by element."""
    from oracle import pmace_oracle as O
    probs = [synth.make_problem(*m) for m in MIX[:4]]
    K = 3
    rule = dict(tol=0.0, min_iter=0, max_iter=K)
    reqs = [serve.Request(i, p, 0.002 * i) for i, p in enumerate(probs)]
    target = 3                                  # Np 128, admitted last
    p = probs[target]
    x0 = synth.make_object(p.n1, p.n2, np.random.default_rng(123))
    reqs[target].x0 = x0.astype(np.complex64)
    ex = serve.GPUExecutor(alpha=0.5, **rule)
    st = serve.Server(ex, 1 << 40, iters_per_step=1, on_step=_tick).run(reqs, serve.FakeClock())
    assert st.completed == len(reqs) and st.max_active > 1
    assert reqs[target].iters == K
    d = p.probe.astype(np.complex64).astype(np.complex128)
    shape = (p.n1, p.n2)
    ost = O.pmace_init(x0.astype(np.complex64).astype(np.complex128), p.pos, p.np_)
    ost = O.pmace_iterate(ost, d, O.amplitudes(p.z.astype(np.float32)), p.pos, shape, 0.5, 1.25, 0.5, K)
    xr = O.reconstruct(ost, d, p.pos, shape, 1.25)
    got = np.asarray(reqs[target].result, np.complex128)
    e = np.linalg.norm(got - xr) / np.linalg.norm(xr)
    m = np.max(np.abs(got - xr)) / np.max(np.abs(xr))
    print(f"  served request vs oracle after {K} iterations: rel {e:.2e} elementwise {m:.2e}", flush=True)
    assert e < 1e-4 and m < 1e-4
