"""Pins of the oracle's data agent F_j (Sec. III-A, eqs. (6)-(9))."""
import numpy as np
import pytest

from conftest import cplx, load_golden
from oracle import pmace_oracle as O
from paper_2111_14240_amd import synth


def _rand_c(rng, shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


@pytest.fixture
def small():
    rng = np.random.default_rng(11)
    np_ = 16
    d = synth.make_probe(np_) * 3.0
    x = _rand_c(rng, (np_, np_))
    y = np.abs(_rand_c(rng, (np_, np_))) * 2.0
    return d, x, y


def test_golden_2x2_cases():
    g = load_golden("agent_2x2_worked.json")
    for case in g["cases"]:
        v = cplx(case["v"])
        d = cplx(case["probe"])
        z = np.asarray(case["z"], float)
        for a, out in case["out"].items():
            got = O.agent(v, d, np.sqrt(z), float(a))
            assert np.allclose(got, cplx(out), atol=1e-12), (case["name"], a, got)


def test_magnitude_step_properties(small):
    d, x, y = small
    W = O.dft2(d * x)
    U = O.fourier_magnitude_step(W, y)
    assert np.allclose(np.abs(U), y)                         # |u| = y where W != 0
    assert np.allclose(np.angle(U[y > 0]), np.angle(W[y > 0]))   # phase kept
    U2 = O.fourier_magnitude_step(U, y)                      # projection: idempotent
    assert np.allclose(U2, U)


def test_magnitude_step_exact_zero():
    W = np.array([[0, 1 + 1j], [0j, -2]])
    y = np.array([[5.0, 2.0], [7.0, 3.0]])
    U = O.fourier_magnitude_step(W, y)
    assert U[0, 0] == 0 and U[1, 0] == 0
    assert np.allclose(U[0, 1], 2 * (1 + 1j) / np.sqrt(2))
    assert np.allclose(U[1, 1], -3)


@pytest.mark.parametrize("alpha", [0.0, 0.3, 1.0, 4.0])
def test_fourier_magnitude_is_r_star(small, alpha):
    """|F D F_j(x)| = (alpha |W| + y)/(1 + alpha) with the phase of W: the r* of
    the first-order condition under eq. (8), a separate statement from eq. (9)."""
    d, x, y = small
    W = O.dft2(d * x)
    out = O.dft2(d * O.agent(x, d, y, alpha))
    assert np.allclose(np.abs(out), (alpha * np.abs(W) + y) / (1 + alpha), atol=1e-10)
    assert np.allclose(out / np.abs(out), W / np.abs(W), atol=1e-10)


def test_alpha_limits(small):
    d, x, y = small
    f0 = O.agent(x, d, y, 0.0)
    assert np.allclose(O.agent(f0, d, y, 0.0), f0, atol=1e-10)   # alpha=0: projection
    assert np.allclose(O.agent(x, d, y, 1e12), x, atol=1e-9)     # alpha -> inf: identity


@pytest.mark.parametrize("alpha", [0.0, 0.5, 2.0])
def test_agent_minimises_eq6(small, alpha):
    """F_j(x) is the minimiser of f_j(v) + ||F D v - F D x||^2/(2 sigma^2); with
    alpha = sigma_n^2/sigma^2 that is 1/2||y - |FDv|||^2 + alpha/2 ||FDv - FDx||^2."""
    d, x, y = small

    def objective(v):
        Wv = O.dft2(d * v)
        return 0.5 * np.sum((y - np.abs(Wv)) ** 2) + 0.5 * alpha * np.sum(
            np.abs(Wv - O.dft2(d * x)) ** 2)

    best = O.agent(x, d, y, alpha)
    f_best = objective(best)
    rng = np.random.default_rng(3)
    for scale in (1e-4, 1e-2, 1.0):
        for _ in range(300):
            assert objective(best + scale * _rand_c(rng, x.shape)) >= f_best - 1e-12


@pytest.mark.parametrize("alpha", [0.0, 0.7, 5.0])
def test_noise_free_truth_is_fixed_point(alpha):
    rng = np.random.default_rng(5)
    np_ = 32
    d = synth.make_probe(np_)
    x = synth.make_object(np_, np_, rng)
    y = np.abs(O.dft2(d * x))
    assert np.allclose(O.agent(x, d, y, alpha), x, atol=1e-10)


def test_zero_probe_pixels_return_input(small):
    d, x, y = small
    d = d.copy()
    d[0, 3] = 0
    d[5, 5] = 0
    out = O.agent(x, d, y, 0.0)
    assert out[0, 3] == x[0, 3] and out[5, 5] == x[5, 5]
    assert np.all(np.isfinite(out))


def test_scale_covariance_of_probe(small):
    """(d, y) -> (c d, |c| y) leaves F_j unchanged (the probe enters through D
    and D^{-1}); a dropped D^{-1} or a conj(d) would break this."""
    d, x, y = small
    c = 0.6 - 1.7j
    assert np.allclose(O.agent(x, c * d, abs(c) * y, 0.4), O.agent(x, d, y, 0.4), atol=1e-10)


def test_data_fit_cost_values():
    """eq. (4): zero at the noise-free truth, sum y^2/(2 sigma_n^2) at v = 0."""
    rng = np.random.default_rng(12)
    d = synth.make_probe(8)
    x = _rand_c(rng, (3, 8, 8))
    y = np.abs(O.dft2(d * x))
    assert O.data_fit_cost(x, d, y) == pytest.approx(0, abs=1e-20)
    assert O.data_fit_cost(np.zeros_like(x), d, y, 2.0) == pytest.approx(np.sum(y ** 2) / 4)


def test_data_fit_cost_scale_by_parseval():
    """eq. (4) with y = 0 is ||F D v||^2 / (2 sigma^2) = ||D v||^2 / (2 sigma^2)
    for the orthonormal F (a missing 1/Np in F would scale it by Np^2), and it
    is quadratic in a common scale of v."""
    rng = np.random.default_rng(13)
    d = synth.make_probe(8)
    v = _rand_c(rng, (2, 8, 8))
    y0 = np.zeros((2, 8, 8))
    assert O.data_fit_cost(v, d, y0, 0.5) == pytest.approx(np.sum(np.abs(d * v) ** 2), rel=1e-12)
    assert O.data_fit_cost(3 * v, d, y0) == pytest.approx(9 * O.data_fit_cost(v, d, y0), rel=1e-12)
