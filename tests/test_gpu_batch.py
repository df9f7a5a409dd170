"""NRMSE (eq. (17)) on the device and batched reconstructions.

The whole iteration is atomic-free with a fixed summation order, so a
reconstruction advanced inside a batch must equal the same reconstruction
advanced alone, bit for bit."""
import sys

import numpy as np
import pytest

from oracle import pmace_oracle as O
from paper_2111_14240_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu-batch]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2111_14240_amd import pmace
    pmace.load_library()
    return pmace


MIX = [  # (n, np, scan, step, peak, seed, chunk)
    (128, 32, 6, 16, None, 1, 0),
    (200, 64, 5, 30, 1e5, 21, 0),
    (160, 64, 4, 28, 1e5, 31, 0),
    (320, 128, 4, 56, 1e5, 22, 0),
    (400, 256, 3, 60, 1e6, 23, 4),
    (300, 256, 2, 40, 1e5, 24, 0),
    (288, 96, 4, 50, 1e5, 25, 0),
    (400, 192, 2, 100, 1e5, 26, 3),
]


def _problems():
    return [synth.make_problem(n, np_, sc, st, pk, sd) for (n, np_, sc, st, pk, sd, _) in MIX]


def _recon(P, prob, chunk, alpha=0.5):
    return P.Reconstruction(prob.n1, prob.n2, prob.probe, prob.pos, prob.z, alpha, chunk=chunk)


def test_nrmse_matches_oracle(P):
    prob = synth.make_problem(160, 64, 4, 28, 1e5, 31)
    mask = synth.roi_mask(prob.probe, prob.pos, prob.n1, prob.n2)
    d = prob.probe.astype(np.complex64).astype(np.complex128)
    shape = (prob.n1, prob.n2)
    st = O.pmace_init(np.ones(shape, complex), prob.pos, prob.np_)
    st = O.pmace_iterate(st, d, O.amplitudes(prob.z), prob.pos, shape, 0.5, 1.25, 0.5, 3)
    ref = O.nrmse(O.reconstruct(st, d, prob.pos, shape, 1.25), prob.x_true, mask)
    _say("nrmse oracle", ref)
    R = _recon(P, prob, 0)
    R.set_state(st.v)
    R.set_reference(prob.x_true, mask)
    e = R.nrmse()
    _say("nrmse device", e)
    assert abs(e - ref) < 1e-5
    R.set_reference(prob.x_true)
    ref_all = O.nrmse(O.reconstruct(st, d, prob.pos, shape, 1.25), prob.x_true)
    assert abs(R.nrmse() - ref_all) < 1e-5
    R.close()


def test_batch_alone_equals_mix_bitwise(P):
    probs = _problems()
    K = 5
    alone = []
    for prob, cfg in zip(probs, MIX):
        _say("alone", cfg)
        R = _recon(P, prob, cfg[-1])
        R.iterate(K)
        alone.append((R.get_state().cpu().numpy(), R.reconstruct().cpu().numpy()))
        R.close()
    _say("mix of", len(probs))
    Rs = [_recon(P, prob, cfg[-1]) for prob, cfg in zip(probs, MIX)]
    B = P.Batch(Rs, tol=0.0, min_iter=0, max_iter=K)
    B.step(K + 3)           # members stop at max_iter; the extra steps must not change them
    done, _, iters = B.poll()
    assert done.tolist() == [1] * len(Rs) and iters.tolist() == [K] * len(Rs)
    for i, R in enumerate(Rs):
        v, xh = R.get_state().cpu().numpy(), R.reconstruct().cpu().numpy()
        assert np.array_equal(v, alone[i][0]) and np.array_equal(xh, alone[i][1]), MIX[i]
    B.close()
    for R in Rs:
        R.close()


def test_batch_large_stage_member_bitwise(P):
    """A row-spectrum member whose stage passes 512 MiB (1089 positions of
    256x256: 558 MiB) takes the batch kernels that write the stage and the new
    states past the caches; advanced in a batch it must equal the same
    reconstruction advanced alone, bit for bit."""
    big = synth.make_problem(768, 256, 33, 15, 1e5, 41)
    small = synth.make_problem(128, 32, 6, 16, None, 1)
    assert big.pos.shape[0] * 256 * 256 * 8 > 512 * 2**20
    K = 3
    alone = []
    for prob in (big, small):
        R = _recon(P, prob, 0)
        if prob is big:
            _say("large-stage member alone, agent", R.agent)
            assert R.agent == "row-spectrum"
        R.iterate(K)
        alone.append((R.get_state().cpu().numpy(), R.reconstruct().cpu().numpy()))
        R.close()
    Rs = [_recon(P, prob, 0) for prob in (big, small)]
    B = P.Batch(Rs, tol=0.0, min_iter=0, max_iter=K)
    B.step(K)
    done, _, iters = B.poll()
    assert done.tolist() == [1, 1] and iters.tolist() == [K, K]
    for i, R in enumerate(Rs):
        v, xh = R.get_state().cpu().numpy(), R.reconstruct().cpu().numpy()
        assert np.array_equal(v, alone[i][0]) and np.array_equal(xh, alone[i][1]), i
    B.close()
    for R in Rs:
        R.close()


def test_batch_stop_rule(P):
    probs = _problems()
    Rs = [_recon(P, prob, cfg[-1]) for prob, cfg in zip(probs, MIX)]
    for R, prob in zip(Rs, probs):
        R.set_reference(prob.x_true, synth.roi_mask(prob.probe, prob.pos, prob.n1, prob.n2))
    B = P.Batch(Rs, tol=2e-3, min_iter=3, max_iter=60)
    steps = 0
    while steps < 80:
        B.step(5)
        steps += 5
        done, nr, iters = B.poll()
        if done.all():
            break
    _say("stop rule: iters", iters.tolist(), "nrmse", np.round(nr, 4).tolist())
    assert done.all()
    assert np.all(iters >= 3) and np.all(iters <= 60)
    # the same rule replayed on each reconstruction advanced alone
    expect = []
    for prob, cfg in zip(probs, MIX):
        A = _recon(P, prob, cfg[-1])
        A.set_reference(prob.x_true, synth.roi_mask(prob.probe, prob.pos, prob.n1, prob.n2))
        prev, k = float("inf"), 0
        while k < 60:
            A.iterate(1)
            k += 1
            e = A.nrmse()
            if k >= 3 and abs(e - prev) < 2e-3:
                break
            prev = e
        expect.append(k)
        A.close()
    _say("stop rule alone: iters", expect)
    assert iters.tolist() == expect
    for R, e in zip(Rs, nr):
        assert abs(R.nrmse() - e) < 1e-12       # the batch's last value is the member's NRMSE
    snap = [R.get_state().cpu().numpy() for R in Rs]
    B.step(3)
    for R, s in zip(Rs, snap):
        assert np.array_equal(R.get_state().cpu().numpy(), s)   # stopped members stay put
    B.close()
    for R in Rs:
        R.close()


def test_stopped_large_member_restarts_when_cleared(P):
    """A poll that finds an Np > 128 member stopped leaves its kernels out of
    the batch's later launches; clearing its flag on the host (pmace_iterate,
    pmace_set_reference) puts it back, inside the captured graph too.  The
    member's history is then 4 batched iterations, 2 alone and the batch's
    iterations up to the rule again: it must equal the same count alone."""
    cases = [(400, 256, 3, 60, 1e6, 23, 4), (400, 192, 2, 100, 1e5, 26, 3), (128, 32, 6, 16, None, 1, 0)]
    probs = [synth.make_problem(n, np_, sc, st, pk, sd) for (n, np_, sc, st, pk, sd, _) in cases]
    Rs = [_recon(P, prob, c[-1]) for prob, c in zip(probs, cases)]
    B = P.Batch(Rs, tol=0.0, min_iter=0, max_iter=4)
    for k in (2, 1, 1):       # the third call runs the captured graph
        B.step(k)
    done, _, iters = B.poll()
    assert done.tolist() == [1, 1, 1] and iters.tolist() == [4, 4, 4]
    _say("cleared member: 4 batched, 2 alone, then the batch again")
    Rs[0].iterate(2)
    B.step(3)                 # one more iteration for member 0 (5 counted >= 4), none for the others
    done, _, iters = B.poll()
    assert done.tolist() == [1, 1, 1] and iters.tolist() == [5, 4, 4]
    Rs[1].set_reference(None)  # counts from zero again: four more batched iterations
    B.step(2)
    B.step(3)
    done, _, iters = B.poll()
    assert done.tolist() == [1, 1, 1] and iters.tolist() == [5, 4, 4]
    for R, prob, c, total in zip(Rs, probs, cases, (7, 8, 4)):
        A = _recon(P, prob, c[-1])
        A.iterate(total)
        same = (np.array_equal(R.get_state().cpu().numpy(), A.get_state().cpu().numpy()) and
                np.array_equal(R.reconstruct().cpu().numpy(), A.reconstruct().cpu().numpy()))
        assert same, (c, total)
        A.close()
    B.close()
    for R in Rs:
        R.close()


FIT_CASES = [  # (n, np, scan, step, peak, seed, chunk)
    (128, 32, 6, 16, 1e5, 41, 0),
    (200, 64, 5, 30, 1e5, 42, 0),
    (320, 128, 4, 56, 1e5, 43, 0),
    (400, 256, 3, 60, 1e6, 44, 4),
    (288, 96, 5, 40, 1e5, 46, 0),
    (360, 160, 3, 80, 1e5, 47, 2),
]


@pytest.mark.parametrize("case", FIT_CASES, ids=lambda c: f"np{c[1]}")
def test_data_fit_matches_oracle(P, case):
    """eq. (4) at the device's current reconstruction, against the oracle's
    cost evaluated at the same reconstruction."""
    n, np_, sc, stp, pk, sd, chunk = case
    prob = synth.make_problem(n, np_, sc, stp, pk, sd)
    R = _recon(P, prob, chunk)
    R.iterate(3)
    R.sync()
    c = R.data_fit()
    xh = R.reconstruct().cpu().numpy().astype(np.complex128)
    d = prob.probe.astype(np.complex64).astype(np.complex128)
    y = O.amplitudes(prob.z.astype(np.float32))
    ref = O.data_fit_cost(O.extract(xh, prob.pos, np_), d, y)
    _say(f"data fit np{np_}: device {c:.8e} oracle {ref:.8e}")
    assert abs(c - ref) <= 1e-4 * ref
    R.close()


def test_data_fit_vanishes_at_noise_free_truth(P):
    prob = synth.make_problem(200, 64, 5, 30, None, 45)
    R = P.Reconstruction(prob.n1, prob.n2, prob.probe, prob.pos, prob.z, 0.5,
                         x0=prob.x_true.astype(np.complex64))
    c = R.data_fit()
    scale = 0.5 * float(np.sum(prob.z))     # the cost at xhat = 0
    _say(f"data fit at the truth {c:.3e} (cost at zero {scale:.3e})")
    assert c <= 1e-9 * scale
    R.close()


def _emulate_fit_rule(P, prob, chunk, tol, min_iter, max_iter, every):
    """The truth-free rule replayed on one reconstruction advanced alone."""
    R = _recon(P, prob, chunk)
    prev, costs = float("inf"), []
    for k in range(1, max_iter + 1):
        R.iterate(1)
        if k % every == 0:
            c = R.data_fit()
            costs.append(c)
            if k >= min_iter and np.isfinite(prev) and abs(c - prev) <= tol * prev:
                R.close()
                return k, c
            prev = c
    R.close()
    return max_iter, (costs[-1] if costs else float("inf"))


def test_batch_data_fit_stop_rule(P):
    probs = _problems()
    tol, min_iter, max_iter, every = 1e-2, 4, 60, 2
    expect = []
    for prob, cfg in zip(probs, MIX):
        expect.append(_emulate_fit_rule(P, prob, cfg[-1], tol, min_iter, max_iter, every))
    _say("data-fit rule, alone:", [e[0] for e in expect])
    assert any(k < max_iter for k, _ in expect)     # the rule itself stops some members
    Rs = [_recon(P, prob, cfg[-1]) for prob, cfg in zip(probs, MIX)]
    B = P.Batch(Rs, tol=tol, min_iter=min_iter, max_iter=max_iter,
                criterion=P.PMACE_STOP_DATA_FIT, check_every=every)
    steps = 0
    while steps < max_iter + 4:
        B.step(4)
        steps += 4
        done, _, iters, fit = B.poll_fit()
        if done.all():
            break
    _say("data-fit rule, batch:", iters.tolist())
    assert done.all()
    assert iters.tolist() == [e[0] for e in expect]
    for (k, c), f in zip(expect, fit):
        assert f == c                        # same kernels, same order: the same value
    B.close()
    for R in Rs:
        R.close()


def test_invalid_stop_rule_rejected(P):
    prob = synth.make_problem(128, 32, 4, 20, None, 3)
    R = _recon(P, prob, 0)
    for kw in (dict(criterion=7), dict(check_every=-1), dict(max_iter=0)):
        with pytest.raises(P.PMACEError) as ei:
            P.Batch([R], **kw)
        assert ei.value.status == P.PMACE_EINVAL
    R.close()


def test_set_stream_moves_a_reconstruction(P):
    """A reconstruction set up on one stream and moved to another (as the
    serving loop does) iterates exactly like one that never moved."""
    prob = synth.make_problem(200, 64, 5, 30, 1e5, 48)
    side, main = torch.cuda.Stream(), torch.cuda.Stream()
    with torch.cuda.stream(side):
        A = P.Reconstruction(prob.n1, prob.n2, prob.probe, prob.pos, prob.z, 0.5, stream=side)
    A.set_stream(main)
    with torch.cuda.stream(main):
        A.iterate(5)
        A.sync()
        va = A.get_state().cpu().numpy()
    B = _recon(P, prob, 0)
    B.iterate(5)
    B.sync()
    assert np.array_equal(va, B.get_state().cpu().numpy())
    A.close()
    B.close()


def test_closing_a_member_of_an_open_batch_is_refused(P):
    prob = synth.make_problem(128, 32, 4, 20, None, 3)
    R = _recon(P, prob, 0)
    B = P.Batch([R])
    with pytest.raises(RuntimeError):
        R.close()
    B.close()
    R.close()


def test_batch_member_new_reference(P):
    """A batched member given a new reference: the batch's stop rule measures
    against the new one (its copy of the member's descriptor is updated)."""
    probs = [synth.make_problem(128, 32, 6, 16, None, 1), synth.make_problem(320, 128, 4, 56, 1e5, 22)]
    Rs = [_recon(P, p, 0) for p in probs]
    for R, p in zip(Rs, probs):
        R.set_reference(p.x_true, synth.roi_mask(p.probe, p.pos, p.n1, p.n2))
    B = P.Batch(Rs, tol=0.0, min_iter=0, max_iter=100)
    B.step(3)
    _, nr0, _ = B.poll()
    # a different reference for member 0 (its object conjugated and scaled),
    # set while the batch holds it
    new_ref = 0.7 * np.conj(probs[0].x_true)
    Rs[0].set_reference(new_ref)
    B.step(1)
    _, nr, iters = B.poll()
    e0 = Rs[0].nrmse()
    _say("new reference: batch", nr[0], "member", e0, "before", nr0[0])
    assert abs(nr[0] - e0) < 1e-12 * max(1.0, abs(e0))
    assert abs(nr[0] - nr0[0]) > 1e-3
    assert abs(nr[1] - Rs[1].nrmse()) < 1e-12
    B.close()
    for R in Rs:
        R.close()


def test_batched_members_match_oracle(P):
    """Members advanced inside a mixed batch (fused sides, a chunked Np = 256
    member on the three-pass agent, the same problem on the row-spectrum
    agent, and an Np = 192 member on the split agent), from smooth starts:
    every member's state and reconstruction after K iterations equal the FP64
    oracle's at 1e-4, in L2 and element by element."""
    # Np 64, 128, 256 (4 positions per chunk) on the three-pass and the
    # row-spectrum agents, 192
    cfgs = [MIX[1], MIX[3], MIX[4], MIX[4], MIX[7]]
    flags = [0, 0, P.PMACE_STAGED_AGENT, P.PMACE_ROWSPEC_AGENT, P.PMACE_SPLIT_AGENT]
    probs = [synth.make_problem(n, np_, sc, st, pk, sd) for (n, np_, sc, st, pk, sd, _) in cfgs]
    K = 3
    x0s = [synth.make_object(p.n1, p.n2, np.random.default_rng(200 + i)).astype(np.complex64)
           for i, p in enumerate(probs)]
    Rs = [P.Reconstruction(p.n1, p.n2, p.probe, p.pos, p.z, 0.5, chunk=cfg[-1], x0=x0, flags=fl)
          for p, cfg, x0, fl in zip(probs, cfgs, x0s, flags)]
    assert [R.agent for R in Rs][2:] == ["three-pass", "row-spectrum", "split"]
    B = P.Batch(Rs, tol=0.0, min_iter=0, max_iter=K)
    B.step(K)
    for i, (R, p) in enumerate(zip(Rs, probs)):
        d = p.probe.astype(np.complex64).astype(np.complex128)
        shape = (p.n1, p.n2)
        st = O.pmace_init(x0s[i].astype(np.complex128), p.pos, p.np_)
        st = O.pmace_iterate(st, d, O.amplitudes(p.z.astype(np.float32)), p.pos, shape, 0.5, 1.25, 0.5, K)
        xr = O.reconstruct(st, d, p.pos, shape, 1.25)
        v, xh = R.get_state().cpu().numpy(), R.reconstruct().cpu().numpy()
        ev = np.linalg.norm(v - st.v) / np.linalg.norm(st.v)
        ex = np.linalg.norm(xh - xr) / np.linalg.norm(xr)
        mv = np.max(np.abs(v - st.v)) / np.max(np.abs(st.v))
        mx = np.max(np.abs(xh - xr)) / np.max(np.abs(xr))
        _say(f"batched member Np {p.np_} ({R.agent}): rel(v)={ev:.2e} rel(xhat)={ex:.2e} "
             f"elementwise {mv:.2e} {mx:.2e}")
        assert ev < 1e-4 and ex < 1e-4 and mv < 1e-4 and mx < 1e-4
    B.close()
    for R in Rs:
        R.close()
