"""Pins of the oracle's SHARP+ (Sec. III-B, eqs. (14)-(15), Alg. 2)."""
import numpy as np
import pytest

from oracle import pmace_oracle as O
from paper_2111_14240_amd import synth


def _prob(seed=2, n=48, np_=16, scan=4, step=8):
    rng = np.random.default_rng(seed)
    x = synth.make_object(n, n, rng)
    d = synth.make_probe(np_) * 1.5
    pos = synth.make_positions(n, np_, scan, step, rng)
    y = np.abs(O.dft2(d * O.extract(x, pos, np_)))
    return x, d, pos, y, rng


def test_projections_are_idempotent():
    x, d, pos, y, rng = _prob()
    s = rng.standard_normal((len(pos), 16, 16)) + 1j * rng.standard_normal((len(pos), 16, 16))
    pa = O.sharp_magnitude_projection(s, y)
    assert np.allclose(O.sharp_magnitude_projection(pa, y), pa, atol=1e-10)
    assert np.allclose(np.abs(O.dft2(pa)), y, atol=1e-10)
    pq = O.sharp_overlap_projection(s, d, pos, x.shape)
    assert np.allclose(O.sharp_overlap_projection(pq, d, pos, x.shape), pq, atol=1e-10)


def test_overlap_projection_keeps_consistent_frames():
    x, d, pos, y, _ = _prob()
    s = d * O.extract(x, pos, 16)
    assert np.allclose(O.sharp_overlap_projection(s, d, pos, x.shape), s, atol=1e-12)
    assert np.allclose(O.sharp_plus_reconstruct(s, d, pos, x.shape)[12:36, 12:36], x[12:36, 12:36])


@pytest.mark.parametrize("beta", [0.3, 0.75, 0.9])
def test_noise_free_truth_is_fixed_point(beta):
    x, d, pos, y, _ = _prob()
    s = d * O.extract(x, pos, 16)
    assert np.allclose(O.sharp_plus_step(s, d, y, pos, x.shape, beta), s, atol=1e-10)


@pytest.mark.parametrize("beta", [0.0, 0.4, 0.8])
def test_step_is_raar_form(beta):
    """Alg. 2's body equals the relaxed averaged alternating reflection
    beta/2 (R_Q R_a + I) + (1 - beta) P_a with R = 2P - I."""
    x, d, pos, y, rng = _prob()
    s = rng.standard_normal((len(pos), 16, 16)) + 1j * rng.standard_normal((len(pos), 16, 16))
    pa = O.sharp_magnitude_projection(s, y)
    ra = 2 * pa - s
    rq_ra = 2 * O.sharp_overlap_projection(ra, d, pos, x.shape) - ra
    raar = 0.5 * beta * (rq_ra + s) + (1 - beta) * pa
    assert np.allclose(O.sharp_plus_step(s, d, y, pos, x.shape, beta), raar, atol=1e-10)


def test_overlap_of_next_state_is_overlap_of_magnitude_step():
    """P_Q s_{k+1} = P_Q P_a s_k (P_Q is a projection): one overlap projection
    per iteration suffices."""
    x, d, pos, y, rng = _prob()
    s = rng.standard_normal((len(pos), 16, 16)) + 1j * rng.standard_normal((len(pos), 16, 16))
    s1 = O.sharp_plus_step(s, d, y, pos, x.shape, 0.7)
    lhs = O.sharp_overlap_projection(s1, d, pos, x.shape)
    rhs = O.sharp_overlap_projection(O.sharp_magnitude_projection(s, y), d, pos, x.shape)
    assert np.allclose(lhs, rhs, atol=1e-10)


def test_init_golden_hand_example():
    """Alg. 2 initialisation s_j = D P_j x0 against the hand-worked example."""
    from conftest import load_golden, cplx
    g = load_golden("sharp_plus_init_worked.json")
    s = O.sharp_plus_init(cplx(g["x0"]), cplx(g["probe"]), np.array(g["pos"]))
    assert s.shape == (2, 2, 2)
    assert np.allclose(s, cplx(g["s"]), rtol=0, atol=1e-15)


@pytest.mark.parametrize("seed", [3, 4])
def test_reconstruct_inverts_init_on_covered_pixels(seed):
    """(sum_k P_k^t |D|^2)^{-1} sum_j P_j^t D^* (D P_j x) = x wherever some
    probe pixel with d != 0 covers the object pixel, and 0 elsewhere."""
    rng = np.random.default_rng(seed)
    n, np_ = 40, 12
    x = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    d = (rng.standard_normal((np_, np_)) + 1j * rng.standard_normal((np_, np_)))
    d[0, :3] = 0.0                     # exact zeros do not cover their pixels
    pos = np.array([[0, 0], [5, 17], [20, 3], [28, 28], [13, 11]])
    s = O.sharp_plus_init(x, d, pos)
    xr = O.sharp_plus_reconstruct(s, d, pos, x.shape)
    cover = O.back_project(np.broadcast_to(np.abs(d) ** 2, (len(pos), np_, np_)), pos, x.shape).real > 0
    assert cover.sum() > 0 and (~cover).sum() > 0
    assert np.allclose(xr[cover], x[cover], rtol=0, atol=1e-12)
    assert np.all(xr[~cover] == 0)
