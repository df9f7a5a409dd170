"""Pins of the measurement simulator reference (eq. (1), eq. (16))."""
import numpy as np
import pytest

from conftest import load_golden
from oracle import pmace_oracle as O
from oracle import simulate_oracle as S
from paper_2111_14240_amd import synth


def test_philox_known_answers():
    for case in load_golden("philox4x32_10_kat.json")["cases"]:
        ctr = [int(v, 16) for v in case["ctr"]]
        key = [int(v, 16) for v in case["key"]]
        assert list(S.philox4x32_10(ctr, key)) == [int(v, 16) for v in case["out"]]


def test_uniforms_open_interval_and_mean():
    u = [S.Uniforms(7, i).next() for i in range(4000)]
    assert 0.0 < min(u) and max(u) < 1.0
    assert abs(np.mean(u) - 0.5) < 5 * np.sqrt(1 / 12 / 4000)


@pytest.mark.parametrize("lam", [0.3, 3.0, 9.9, 10.0, 57.0, 1000.0, 1e5])
def test_poisson_moments(lam):
    n = 3000
    x = S.poisson(np.full(n, lam), seed=11)
    assert np.all(x == np.round(x)) and x.min() >= 0
    m, v = x.mean(), x.var()
    assert abs(m - lam) < 5 * np.sqrt(lam / n)                 # mean
    assert abs(v / lam - 1) < 5 * np.sqrt(2 / n) + 0.02        # variance = mean


def test_poisson_small_mean_pmf():
    lam, n = 2.0, 4000
    x = S.poisson(np.full(n, lam), seed=3).astype(int)
    import math
    for k in range(5):
        p = math.exp(-lam) * lam ** k / math.factorial(k)
        assert abs(np.mean(x == k) - p) < 5 * np.sqrt(p * (1 - p) / n)


def test_forward_model_matches_generator_and_energy():
    p = synth.make_config_problem("c1")
    inten = S.forward_intensities(p.x_true, p.probe, p.pos)
    assert np.allclose(inten, p.z, rtol=1e-5, atol=1e-6)        # synth's noise-free data
    for j in (0, 20):
        r, c = p.pos[j]
        e = np.sum(np.abs(p.probe * p.x_true[r:r + 32, c:c + 32]) ** 2)
        assert inten[j].sum() == pytest.approx(e, rel=1e-12)    # Parseval
    # the noise-free truth is a fixed point of the agent with y = sqrt(I)
    xj = p.x_true[p.pos[5][0]:p.pos[5][0] + 32, p.pos[5][1]:p.pos[5][1] + 32]
    assert np.allclose(O.agent(xj, p.probe, np.sqrt(inten[5]), 0.3), xj, atol=1e-10)


def test_simulate_scaling():
    p = synth.make_problem(48, 16, 3, 12, None, seed=4)
    z, scale = S.simulate(p.x_true, p.probe, p.pos, 500.0, seed=9)
    inten = S.forward_intensities(p.x_true, p.probe, p.pos)
    assert scale == pytest.approx(500.0 / inten.max())
    assert abs(z.sum() / (inten.sum() * scale) - 1) < 0.02
    z2, _ = S.simulate(p.x_true, p.probe, p.pos, 500.0, seed=9)
    assert np.array_equal(z, z2)
