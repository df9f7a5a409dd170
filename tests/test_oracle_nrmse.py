"""Pins of the oracle's NRMSE (eq. (17)) and of the synthetic input generator."""
import numpy as np
import pytest

from oracle import pmace_oracle as O
from paper_2111_14240_amd import synth


def test_nrmse_special_values():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((20, 20)) + 1j * rng.standard_normal((20, 20))
    assert O.nrmse(np.exp(2.2j) * x, x) == pytest.approx(0, abs=1e-14)
    assert O.nrmse(np.zeros_like(x), x) == pytest.approx(1.0)
    assert O.nrmse(2 * x, x) == pytest.approx(1.0)


def test_nrmse_theta_is_grid_minimiser():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((16, 16)) + 1j * rng.standard_normal((16, 16))
    xh = np.exp(0.77j) * x + 0.3 * (rng.standard_normal(x.shape) + 1j * rng.standard_normal(x.shape))
    thetas = np.linspace(0, 2 * np.pi, 10000, endpoint=False)
    grid = min(np.linalg.norm(xh - np.exp(1j * t) * x) for t in thetas) / np.linalg.norm(x)
    e = O.nrmse(xh, x)
    assert e <= grid + 1e-12
    assert e == pytest.approx(grid, abs=1e-6)


def test_nrmse_mask():
    x = np.ones((4, 4), complex)
    xh = x.copy()
    xh[0, 0] = 100
    m = np.ones((4, 4), bool)
    m[0, 0] = False
    assert O.nrmse(xh, x, m) == pytest.approx(0, abs=1e-14)


def test_generator_is_deterministic_and_in_range():
    a = synth.make_config_problem("c1")
    b = synth.make_config_problem("c1")
    assert np.array_equal(a.z, b.z) and np.array_equal(a.pos, b.pos)
    assert np.array_equal(a.x_true, b.x_true)
    mag = np.abs(a.x_true)
    ph = np.angle(a.x_true)
    assert mag.min() >= 0.5 - 1e-12 and mag.max() <= 1 + 1e-12
    assert ph.min() >= -np.pi / 2 - 1e-12 and ph.max() <= np.pi / 2 + 1e-12
    assert a.pos.min() >= 0 and a.pos.max() <= a.n1 - a.np_
    assert a.pos.shape == (36, 2) and a.z.shape == (36, 32, 32)


def test_positions_centred_jittered_clamped():
    rng = np.random.default_rng(3)
    pos = synth.make_positions(1024, 256, 40, 20, rng)
    assert pos.min() == 0 and pos.max() == 1024 - 256
    base = (1024 - (39 * 20 + 256)) // 2 + 20 * np.arange(40)
    r = pos[:, 0].reshape(40, 40)[:, 0]
    inner = (base >= 2) & (base <= 1024 - 256 - 2)
    assert np.all(np.abs(r[inner] - base[inner]) <= 2)


def test_noise_free_intensity_energy():
    """Orthonormal F preserves energy: sum_p z_j = sum_p |d P_j x|^2 (eq. (1))."""
    p = synth.make_config_problem("c1")
    for j in (0, 17, 35):
        r, c = p.pos[j]
        e = np.sum(np.abs(p.probe * p.x_true[r:r + 32, c:c + 32]) ** 2)
        assert p.z[j].sum() == pytest.approx(e, rel=1e-5)


def test_poisson_peak_scaling():
    p = synth.make_problem(64, 16, 4, 8, 1e4, seed=9)
    lam = np.stack([np.abs(np.fft.fft2(p.probe * p.x_true[r:r + 16, c:c + 16], norm="ortho")) ** 2
                    for r, c in p.pos])
    assert lam.max() == pytest.approx(1e4, rel=1e-9)
    assert np.all(p.z == np.round(p.z)) and p.z.min() >= 0
    assert abs(p.z.sum() / lam.sum() - 1) < 0.01


def test_mix_specs_fit():
    specs = synth.draw_mix_specs()
    assert len(specs) == 64
    for s in specs:
        assert s["np_"] <= s["n"] // 2
        assert (s["scan"] - 1) * s["step"] + s["np_"] <= s["n"] - 4 or s["step"] == 1
        assert s["step"] <= s["np_"] // 2
