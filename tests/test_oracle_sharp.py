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
