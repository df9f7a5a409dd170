"""Pins of the oracle's Algorithm 1 (Mann iteration of T = (2G-I)(2F-I))."""
import numpy as np
import pytest

from conftest import cplx, load_golden
from oracle import pmace_oracle as O
from paper_2111_14240_amd import synth


def _noise_free(seed=3, n=48, np_=16, scan=4, step=8):
    rng = np.random.default_rng(seed)
    x = synth.make_object(n, n, rng)
    d = synth.make_probe(np_) * 2.0
    pos = synth.make_positions(n, np_, scan, step, rng)
    y = np.abs(O.dft2(d * O.extract(x, pos, np_)))
    return x, d, pos, y


def test_golden_worked_two_iterations():
    g = load_golden("alg1_np1_worked.json")
    x0 = cplx(g["x0"])
    d = cplx(g["probe"])
    pos = np.asarray(g["pos"])
    y = O.amplitudes(np.asarray(g["z"], float))
    st = O.pmace_init(x0, pos, 1)
    shape = x0.shape
    for it in ("iter1", "iter2"):
        st = O.pmace_iterate(st, d, y, pos, shape, g["alpha"], g["kappa"], g["rho"], 1)
        ref = g[it]
        assert np.allclose(st.w[:, 0, 0], cplx(ref["w"]), atol=1e-12), it
        assert np.allclose(st.z[:, 0, 0], cplx(ref["z"]), atol=1e-12), it
        assert np.allclose(st.v[:, 0, 0], cplx(ref["v"]), atol=1e-12), it
        xh = O.reconstruct(st, d, pos, shape, g["kappa"])
        assert np.allclose(xh[0], cplx(ref["xhat"]), atol=1e-12), it


@pytest.mark.parametrize("alpha,kappa,rho", [(0.0, 1.25, 0.5), (0.8, 2.0, 0.3), (3.0, 0.5, 0.9)])
def test_noise_free_truth_is_fixed_point(alpha, kappa, rho):
    x, d, pos, y = _noise_free()
    v = O.extract(x, pos, d.shape[0])
    v1, w, z = O.pmace_step(v, d, y, pos, x.shape, alpha, kappa, rho)
    assert np.allclose(w, v, atol=1e-10)
    assert np.allclose(z, w, atol=1e-10)
    assert np.allclose(v1, v, atol=1e-10)


def test_step_equals_mann_update_of_T():
    """Alg. 1's loop body equals x <- (1-rho) x + rho T x (eqs. (12)-(13))."""
    rng = np.random.default_rng(4)
    x, d, pos, y = _noise_free()
    y = y * (1 + 0.2 * rng.random(y.shape))
    v = O.extract(x, pos, d.shape[0]) * np.exp(0.3j) + 0.1
    for rho in (0.25, 0.5, 0.8):
        v1, _, _ = O.pmace_step(v, d, y, pos, x.shape, 0.6, 1.25, rho)
        mann = (1 - rho) * v + rho * O.T_operator(v, d, y, pos, x.shape, 0.6, 1.25)
        assert np.allclose(v1, mann, atol=1e-12)


def test_non_overlapping_half_step_is_agent():
    """With G = I (no overlap) and rho = 1/2 the loop body reduces to v <- F(v)."""
    rng = np.random.default_rng(6)
    np_ = 8
    d = synth.make_probe(np_)
    pos = np.array([[0, 0], [0, 8], [8, 0], [8, 8]])
    v = rng.standard_normal((4, np_, np_)) + 1j * rng.standard_normal((4, np_, np_))
    y = np.abs(rng.standard_normal((4, np_, np_)))
    v1, w, _ = O.pmace_step(v, d, y, pos, (16, 16), 0.3, 1.25, 0.5)
    assert np.allclose(v1, O.agent_stack(v, d, y, 0.3), atol=1e-12)


def test_equivariances():
    rng = np.random.default_rng(8)
    x, d, pos, y = _noise_free()
    y = y * (1 + 0.3 * rng.random(y.shape))
    x0 = np.ones(x.shape, complex)
    args = (0.5, 1.25, 0.5)
    ref = O.pmace_iterate(O.pmace_init(x0, pos, d.shape[0]), d, y, pos, x.shape, *args, 3)
    # global phase of the start
    ph = np.exp(1.1j)
    st = O.pmace_iterate(O.pmace_init(ph * x0, pos, d.shape[0]), d, y, pos, x.shape, *args, 3)
    assert np.allclose(st.v, ph * ref.v, atol=1e-10)
    # probe and data scaling (d, z) -> (c d, |c|^2 z)
    c = 1.7 - 0.4j
    st = O.pmace_iterate(O.pmace_init(x0, pos, d.shape[0]), c * d, abs(c) * y, pos, x.shape, *args, 3)
    assert np.allclose(st.v, ref.v, atol=1e-10)
    # integer translation of the object grid and every position
    big = np.ones((x.shape[0] + 5, x.shape[1] + 9), complex)
    st = O.pmace_iterate(O.pmace_init(big, pos + np.array([5, 9]), d.shape[0]), d, y,
                         pos + np.array([5, 9]), big.shape, *args, 3)
    assert np.allclose(st.v, ref.v, atol=1e-10)


def test_image_recurrence_matches_direct_average():
    """xhat_{k+1} = (1-rho) xhat_k + rho xbar_k, xbar_k = weighted average of 2w - v."""
    rng = np.random.default_rng(9)
    x, d, pos, y = _noise_free()
    y = y * (1 + 0.3 * rng.random(y.shape))
    shape, kap, rho = x.shape, 1.25, 0.5
    lam = O.weight_image(d, pos, shape, kap)
    st = O.pmace_init(np.ones(shape, complex), pos, d.shape[0])
    xh = O.reconstruct(st, d, pos, shape, kap)
    assert np.allclose(xh[lam > 0], 1.0)
    for _ in range(4):
        v = st.v
        st = O.pmace_iterate(st, d, y, pos, shape, 0.5, kap, rho, 1)
        xbar = O.weighted_average(2 * st.w - v, d, pos, shape, kap)
        xh = (1 - rho) * xh + rho * xbar
        assert np.allclose(xh, O.reconstruct(st, d, pos, shape, kap), atol=1e-12)


def test_converges_on_noise_free_small_problem():
    x, d, pos, y = _noise_free(n=40, np_=16, scan=5, step=6)
    mask = synth.roi_mask(d, pos, *x.shape)
    xh, st, h = O.pmace_solve(np.ones(x.shape, complex), d, y ** 2, pos, 0.05, 1.25, 0.5, 60,
                              x_true=x, mask=mask)
    e = h["nrmse"]
    assert e[-1] < 0.5 * e[0]
    # at convergence z -> w (fixed point of T gives G(2w - v) = w)
    rel = np.linalg.norm(st.z - st.w) / np.linalg.norm(st.w)
    assert rel < 0.05
