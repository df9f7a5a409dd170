"""Device measurement simulator (eq. (1), eq. (16)) against its reference."""
import sys

import numpy as np
import pytest

from conftest import load_golden
from oracle import simulate_oracle as S
from paper_2111_14240_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu-sim]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2111_14240_amd import pmace
    pmace.load_library()
    return pmace


def test_philox_known_answers_on_device(P):
    cases = load_golden("philox4x32_10_kat.json")["cases"]
    rec = np.array([[int(v, 16) for v in c["ctr"] + c["key"]] for c in cases], dtype=np.uint32)
    out = P.philox4x32_10(rec)
    assert out.tolist() == [[int(v, 16) for v in c["out"]] for c in cases]


def test_poisson_sampler_matches_reference(P):
    rng = np.random.default_rng(0)
    lam = np.concatenate([rng.uniform(0, 10, 1500), rng.uniform(10, 200, 1500),
                          rng.uniform(1e3, 1e6, 1000), [0.0, 9.999999, 10.0]])
    _say("poisson", lam.size)
    got = P.poisson(lam, seed=1234)
    ref = S.poisson(lam, seed=1234)
    same = np.mean(got == ref)
    _say("identical draws", same)
    assert same >= 0.999     # FP64 log/lgamma of the two libraries may flip a boundary draw
    assert np.all(np.abs(got - ref)[got != ref] <= 2)


@pytest.mark.parametrize("np_,peak", [(32, None), (64, 1e5), (96, None), (128, 1e4), (160, 1e5),
                                      (256, 1e6)])
def test_simulate_matches_reference(P, np_, peak):
    prob = synth.make_problem(np_ * 2, np_, 3, np_ // 3, None, seed=40 + np_)
    x = prob.x_true.astype(np.complex64).astype(np.complex128)
    d = prob.probe.astype(np.complex64).astype(np.complex128)
    _say("simulate", np_, peak)
    z, scale = P.simulate(x, d, prob.pos, peak, seed=77)
    z = z.cpu().numpy()
    inten = S.forward_intensities(x, d, prob.pos)
    if peak is None:
        assert scale == 1.0
        assert np.linalg.norm(z - inten) / np.linalg.norm(inten) < 2e-6
    else:
        assert scale == pytest.approx(peak / inten.max(), rel=1e-5)
        assert np.all(z == np.round(z)) and z.min() >= 0
        lam = inten * scale
        assert abs(z.sum() / lam.sum() - 1) < 5 / np.sqrt(lam.sum())
        z2, _ = P.simulate(x, d, prob.pos, peak, seed=77)
        assert np.array_equal(z, z2.cpu().numpy())          # reproducible
        sub = slice(0, 2000)
        ref = S.poisson(lam.ravel()[sub], seed=77)
        assert np.mean(z.ravel()[sub] == ref) >= 0.99        # same streams, FP32 vs FP64 means


def test_simulate_into_caller_buffers(P):
    """Caller-owned output and workspace (reused across calls, stale
    contents left in both) give exactly the freshly allocated call's counts;
    a wrong output shape is refused before anything runs."""
    prob = synth.make_problem(320, 128, 4, 60, None, seed=91)
    dev = torch.device("cuda")
    ref, s_ref = P.simulate(prob.x_true, prob.probe, prob.pos, 1e5, seed=5)
    fp = int(P.load_library().pmace_simulate_footprint(128, len(prob.pos)))
    ws = torch.full((fp,), 0xAB, dtype=torch.uint8, device=dev)
    out = torch.full((len(prob.pos), 128, 128), -1.0, dtype=torch.float32, device=dev)
    _say("simulate into caller buffers, twice")
    for _ in range(2):
        z, s = P.simulate(prob.x_true, prob.probe, prob.pos, 1e5, seed=5, out=out, workspace=ws)
        assert z.data_ptr() == out.data_ptr() and s == s_ref
        assert torch.equal(z, ref)
    with pytest.raises(ValueError):
        P.simulate(prob.x_true, prob.probe, prob.pos, 1e5, seed=5, out=out[:-1], workspace=ws)
    with pytest.raises(ValueError):
        P.simulate(prob.x_true, prob.probe, prob.pos, 1e5, seed=5, out=out, workspace=ws[:16])


@pytest.mark.slow
def test_simulate_c3_geometry_full_size(P):
    """The simulator as bench.py --mode simulate runs it: the C3 geometry
    (1024^2 object, 1600 positions of 256^2, peak 1e6).  Noise-free
    intensities on every frame against the oracle's forward model; the photon
    scale of eq. (16) against the oracle's global maximum; Poisson counts on
    sampled elements against the oracle's sampler on the same streams."""
    c = synth.CONFIGS["c3"]
    rng = np.random.default_rng(c["seed"])
    n, np_ = c["n"], c["np_"]
    x = synth.make_object(n, n, rng).astype(np.complex64).astype(np.complex128)
    d = synth.make_probe(np_).astype(np.complex64).astype(np.complex128)
    pos = synth.make_positions(n, np_, c["scan"], c["step"], rng)
    _say("simulate c3 geometry: oracle intensities")
    inten = S.forward_intensities(x, d, pos)
    z0, s0 = P.simulate(x, d, pos, None, seed=3)
    assert s0 == 1.0
    e = np.linalg.norm(z0.cpu().numpy() - inten) / np.linalg.norm(inten)
    _say(f"  noise-free rel {e:.2e}")
    assert e < 2e-6
    z, scale = P.simulate(x, d, pos, 1e6, seed=3)
    assert scale == pytest.approx(1e6 / inten.max(), rel=1e-5)
    zc = z.cpu().numpy().ravel()
    lam = (inten * scale).ravel()
    pick = np.random.default_rng(1).choice(lam.size, 3000, replace=False)
    pick.sort()
    # the oracle's streams are counted by element index, so each sampled element
    # is drawn from its own stream
    ref = np.array([S.poisson_draw(float(lam[i]), S.Uniforms(3, int(i))) for i in pick])
    same = np.mean(zc[pick] == ref)
    _say(f"  sampled counts equal: {same:.4f}")
    assert same >= 0.99
