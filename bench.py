"""PMACE throughput on one MI355X.

One step = one iteration of the PMACE loop body over every scan position of
the workload (agent F_j on all patches, consensus G, Mann update, image
recurrence), with all inputs resident in HBM.  Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--config c3]
  python bench.py --method sharp [--beta 0.8]      SHARP+ (Alg. 2) on the same workload
  python bench.py --np 192                         the workload with another probe side
  python bench.py --mode simulate                  the device measurement simulator (eq. (1), (16))
  python bench.py --mode batch [--items 64]        mixed-size batch vs plain, same stop rule
  python bench.py --mode serve [--requests 2000]   continuous batching vs plain FIFO
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "pmace_hbm_traffic.md")
KERNEL_SOURCES = ["csrc/pmace_kernels.hip", "csrc/pmace_dft.hpp", "csrc/pmace_internal.hpp",
                  "csrc/pmace_api.hip", "tuned.json"]
FP32_VECTOR_PEAK_TFLOPS = 157.3
# What `traffic` counts: requests leaving the L2 for the memory fabric
# (FETCH_SIZE + WRITE_SIZE, each scaled by the same counter on a plain copy).
# The Infinity Cache sits behind those requests, so its hits are included.
TRAFFIC_LEVEL = "L2-to-fabric bytes per iteration (Infinity Cache hits included)"
ALPHA = {"c1": 0.1, "c2": 0.5, "c3": 0.5}


def algorithmic_bytes(J, np_, n1, n2):
    """Per iteration: read state 8 B + amplitudes 4 B, write state 8 B per
    patch pixel; read numerator 8 B + Lambda^{-1} 4 B, write xbar 8 B per
    object pixel.  SHARP+ (Alg. 2) is counted the same way: its state is the
    frame s_j, and the overlap projection's sums are object-sized."""
    return 20.0 * J * np_ * np_ + 20.0 * n1 * n2


def algorithmic_flops(J, np_):
    """Two 2-D FFTs (5 N log2 N per 1-D transform) + 36 pointwise flops per patch pixel."""
    return J * np_ * np_ * (20.0 * np.log2(np_) + 36.0)


def kernel_source_hash():
    """Hash of the sources and the tuned build defines the iteration kernels are
    built from (of tuned.json only its "defines": the timings it records do not
    change the build)."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        path = os.path.join(ROOT, "paper_2111_14240_amd", f)
        if not os.path.exists(path):
            continue
        if f == "tuned.json":
            with open(path) as fh:
                h.update(json.dumps(json.load(fh).get("defines", {}), sort_keys=True).encode())
        else:
            with open(path, "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()[:16]


def iteration_kernels(np_, J, method="pmace", agent="three-pass"):
    """The kernels one timed iteration (the roofline's unit) launches, for the
    agent the reconstruction runs ('whole patch', 'three-pass', 'split',
    'row-spectrum')."""
    name = "PMACE" if method == "pmace" else "SHARP+"
    if agent == "split":
        return (f"one {name} iteration: agent_split_pair<{np_ // 2}> ({2 * J} workgroups, two "
                f"{np_ // 2}x{np_ // 2} coset blocks each) + consensus_split<{np_ // 2}> (four partial sums "
                f"per pixel) + image_update_split")
    if agent == "row-spectrum":
        return (f"one {name} iteration: per chunk of positions agent_rows, agent_cols <{np_}> "
                f"(states kept as row spectra) + consensus_rows<{np_}> (inverse row DFTs, one object "
                f"row per workgroup; a9 fused when one chunk holds every position, else image_update "
                f"after the last chunk)")
    if np_ <= 128:
        return (f"one {name} iteration: agent_fused<{np_}> ({J} workgroups) + "
                f"consensus_gather<{np_}> (a9 fused)")
    return (f"one {name} iteration: per chunk of positions agent_rows, agent_cols, "
            f"agent_rowsinv <{np_}> + consensus_gather<{np_}>, then image_update")


def raster_overhang(n, np_, scan, step):
    """Note for a centred raster wider than the object: its edge positions are
    clamped to the object (so the outermost steps are shorter)."""
    ov = (scan - 1) * step + np_ - n
    return f"; the raster overhangs the object by {ov} px, edge rows and columns clamped" if ov > 0 else ""


def workload_key(config, method, np_override, agent="default"):
    """Row name of a workload in the traffic table: the config, then the
    variant ('c3', 'c3-sharp', 'c3-np192', 'c3-staged')."""
    key = config
    if method != "pmace":
        key += "-" + method
    if np_override:
        key += f"-np{np_override}"
    if agent != "default":
        key += "-" + agent
    return key


def measured_traffic(config):
    """HBM bytes per iteration measured with rocprofv3 counters (FETCH_SIZE and
    WRITE_SIZE, each scaled by the same counter on a plain copy of known size),
    or None if not measured for the current kernel sources.  Read from the
    table row '| <config> | <source hash> | ... | <bytes per iteration> |'."""
    try:
        with open(TRAFFIC_FILE) as f:
            lines = f.read().splitlines()
    except OSError:
        return None
    h = kernel_source_hash()
    for ln in lines:
        cells = [c.strip() for c in ln.strip().strip("|").split("|")]
        if len(cells) >= 3 and cells[0] == config and cells[1] == h:
            try:
                return float(cells[-1])
            except ValueError:
                return None
    return None


def calibration_copy(mib):
    """A plain device copy of known size (outside any timed region) whose
    FETCH_SIZE / WRITE_SIZE calibrate the counters."""
    import torch
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()


def cpu_model():
    """The host CPU's model name (from /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline_all_cores(prob, alpha, kappa, rho, min_seconds=10.0, max_iters=6, method="pmace", beta=0.0):
    """The same oracle with its FFT primitive (numpy's, one thread) served by
    scipy.fft on every host core: the oracle's own arithmetic is unchanged,
    only the library transform runs multi-threaded."""
    import scipy.fft as sf
    from oracle import pmace_oracle as O
    cores = os.cpu_count() or 1
    saved = (O.dft2, O.idft2)
    O.dft2 = lambda a: sf.fft2(np.asarray(a, dtype=np.complex128), norm="ortho", workers=cores)
    O.idft2 = lambda a: sf.ifft2(np.asarray(a, dtype=np.complex128), norm="ortho", workers=cores)
    try:
        out = cpu_baseline(prob, alpha, kappa, rho, min_seconds, max_iters, method, beta)
    finally:
        O.dft2, O.idft2 = saved
    out["cores"] = cores
    out["sample"] = out["sample"].replace("numpy FFT (single thread)",
                                          f"scipy.fft on {cores} threads for the transforms")
    return out


def cpu_baseline(prob, alpha, kappa, rho, min_seconds=12.0, max_iters=6, method="pmace", beta=0.0):
    """The FP64 oracle, as it stands, timed on whole iterations of the same
    workload until at least min_seconds have passed (at most max_iters)."""
    from oracle import pmace_oracle as O
    d = prob.probe.astype(np.complex64).astype(np.complex128)
    y = O.amplitudes(prob.z)
    shape = (prob.n1, prob.n2)
    x0 = np.ones(shape, complex)
    if method == "pmace":
        st = O.pmace_init(x0, prob.pos, prob.np_)
        step = lambda st: O.pmace_iterate(st, d, y, prob.pos, shape, alpha, kappa, rho, 1)
    else:
        st = O.sharp_plus_init(x0, d, prob.pos)
        step = lambda st: O.sharp_plus_step(st, d, y, prob.pos, shape, beta)
    k, t0 = 0, time.perf_counter()
    while True:
        st = step(st)
        k += 1
        dt = time.perf_counter() - t0
        if dt >= min_seconds or k >= max_iters:
            break
    return {"value": k * prob.num_pos / dt, "unit": "patch-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"{k} iterations of the full workload ({prob.num_pos} positions each), "
                      f"{dt:.2f} s, numpy FFT (single thread)",
            "cpu_model": cpu_model(), "host_cpu_count": os.cpu_count()}


_MIX_CACHE = {}


def _mix_problems(count, seed=4, device="cuda"):
    """The mixed-size workload: sizes from the seeded draw, intensities
    simulated on the device (Poisson peak 1e5); made once per process."""
    from paper_2111_14240_amd import pmace, synth
    key = (count, seed, str(device))
    if key not in _MIX_CACHE:
        specs = synth.draw_mix_specs(count, seed=seed)
        _MIX_CACHE[key] = [pmace.simulated_problem(s["n"], s["np_"], s["scan"], s["step"], s["peak"], s["seed"],
                                                   device=device) for s in specs]
    return _MIX_CACHE[key]


def _stop_rule(args):
    """NRMSE change < 1e-4 (eq. (17), needs the synthetic truth), or the
    truth-free relative change of the data-fit cost (eq. (4))."""
    from paper_2111_14240_amd import pmace
    if args.stop == "data_fit":
        return dict(tol=args.fit_tol, min_iter=2, max_iter=500, criterion=pmace.PMACE_STOP_DATA_FIT,
                    check_every=args.check_every)
    return dict(tol=1e-4, min_iter=2, max_iter=500, criterion=pmace.PMACE_STOP_NRMSE,
                check_every=args.check_every)


def bench_batch(args):
    print(json.dumps(batch_comparison(args)), flush=True)


def batch_comparison(args):
    """All reconstructions advanced together (one graph launch per iteration)
    versus the plain solver (one at a time, in order), both to the same
    on-device stop rule; alone and in the batch each member takes the same
    iterations and ends at the same NRMSE (the path is deterministic)."""
    import torch
    from paper_2111_14240_amd import pmace, synth
    t0 = time.perf_counter()
    probs = _mix_problems(args.items)
    torch.cuda.synchronize()
    gen_s = time.perf_counter() - t0
    alpha = 0.5
    rule = _stop_rule(args)
    poll = 10

    def make(p):
        R = pmace.Reconstruction(p.n1, p.n2, p.probe, p.pos, p.z, alpha)
        R.set_reference(p.x_true, synth.roi_mask(p.probe, p.pos, p.n1, p.n2))
        return R

    def drive(B, n):
        steps = 0
        while True:
            B.step(poll)
            steps += poll
            done, nr, it = B.poll()
            if done.all() or steps > rule["max_iter"] + poll:
                return nr, it

    # plain: one reconstruction at a time
    plain_nr, plain_it = [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    on_demand = args.stop != "nrmse"   # the rule does not track NRMSE: measure it at the end
    for p in probs:
        R = make(p)
        B = pmace.Batch([R], **rule)
        nr, it = drive(B, 1)
        plain_nr.append(R.nrmse() if on_demand else nr[0])
        plain_it.append(it[0])
        B.close()
        R.close()
    torch.cuda.synchronize()
    plain_s = time.perf_counter() - t0
    # batched
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Rs = [make(p) for p in probs]
    B = pmace.Batch(Rs, **rule)
    nr, it = drive(B, len(Rs))
    torch.cuda.synchronize()
    batch_s = time.perf_counter() - t0
    if on_demand:
        nr = np.array([R.nrmse() for R in Rs])
    B.close()
    for R in Rs:
        R.close()
    patch_updates = float(sum(p.num_pos * k for p, k in zip(probs, it)))
    B_alg = sum(algorithmic_bytes(p.num_pos, p.np_, p.n1, p.n2) * k for p, k in zip(probs, it))
    out = {
        "metric": "batched-vs-plain solves/s",
        "value": len(probs) / batch_s, "unit": "solves/s", "n_gpus": 1,
        "higher_is_better": True, "vs_baseline": None, "dtype": "c64", "data": "synthetic (simulated on device)",
        "config": {"workload": f"{len(probs)} reconstructions, object {{256,512,1024}}, probe {{64,128,256}}, "
                               "scan 7x7..30x30, Poisson peak 1e5", "stop_rule": rule, "alpha": alpha,
                   "poll_every": poll},
        "batched": {"seconds": batch_s, "solves_per_s": len(probs) / batch_s,
                    "patch_updates_per_s": patch_updates / batch_s,
                    "algorithmic_GBps": B_alg / batch_s / 1e9},
        "plain": {"seconds": plain_s, "solves_per_s": len(probs) / plain_s,
                  "patch_updates_per_s": patch_updates / plain_s},
        "speedup": plain_s / batch_s,
        "same_iterations": [int(a) for a in plain_it] == [int(b) for b in it],
        "same_nrmse": bool(np.array_equal(np.asarray(plain_nr), np.asarray(nr))),
        "iterations": {"min": int(min(it)), "median": float(np.median(it)), "max": int(max(it))},
        "nrmse": {"median": float(np.median(nr)), "max": float(np.max(nr))},
        "generation_s": gen_s,
        "total_patch_pixels": int(sum(p.patch_pixels for p in probs)),
    }
    return out


def simulate_cpu_baseline(x, d, pos, peak, seed, min_seconds=10.0):
    """The oracle's simulator (forward model, Philox4x32-10, Poisson draws in
    plain Python) on the first k frames of the workload, k sized from one
    timed frame so the sample takes about min_seconds; the photon scale of
    eq. (16) is taken over the sample."""
    from oracle import simulate_oracle as SO
    t0 = time.perf_counter()
    SO.simulate(x, d, pos[:1], peak, seed)
    one = time.perf_counter() - t0
    k = int(min(len(pos), max(1, np.ceil(min_seconds / max(one, 1e-9)))))
    t0 = time.perf_counter()
    SO.simulate(x, d, pos[:k], peak, seed)
    dt = time.perf_counter() - t0
    return {"value": k / dt, "unit": "frames/s", "cores": 1, "kind": "oracle",
            "sample": f"the first {k} frames of the workload ({d.shape[0]}x{d.shape[0]}), {dt:.2f} s, "
                      "numpy FFT, Poisson draws in plain Python (single thread)"}


def bench_simulate(args):
    """The measurement simulator of eq. (1) and eq. (16) on the workload's
    geometry: frames d P_j x, 2-D DFTs, intensities and their maximum, Poisson
    draws.  One step = one pmace_simulate call over every position (it
    synchronises twice: positions are checked on the host, the photon scale is
    read back)."""
    import torch
    from paper_2111_14240_amd import pmace, synth
    cfg = dict(synth.CONFIGS[args.config])
    if args.np:
        cfg["np_"] = args.np
    peak = cfg["peak"] or 1e5
    rng = np.random.default_rng(cfg["seed"])
    n, np_ = cfg["n"], cfg["np_"]
    x = synth.make_object(n, n, rng)
    d = synth.make_probe(np_)
    pos = synth.make_positions(n, np_, cfg["scan"], cfg["step"], rng)
    J = len(pos)
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(device=dev)
    x_t = pmace.to_device_c64(x, dev)
    d_t = pmace.to_device_c64(d, dev)
    pos_t = torch.as_tensor(pos, dtype=torch.int32).to(dev)
    z = torch.empty((J, np_, np_), dtype=torch.float32, device=dev)
    ws = torch.empty(int(pmace.load_library().pmace_simulate_footprint(np_, J)), dtype=torch.uint8,
                     device=dev)
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        for i in range(args.warmup):
            pmace.simulate(x_t, d_t, pos_t, peak, 1000 + i, device=dev, stream=stream, out=z, workspace=ws)
        torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        ev0.record(stream)
        for i in range(args.steps):
            _, scale = pmace.simulate(x_t, d_t, pos_t, peak, 2000 + i, device=dev, stream=stream, out=z,
                                      workspace=ws)
        ev1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        gpu_ms = ev0.elapsed_time(ev1)
    ms = gpu_ms / args.steps
    # algorithmic bytes: the object and probe read once, the counts written once
    B = 8.0 * n * n + 8.0 * np_ * np_ + 4.0 * J * np_ * np_
    achieved = B / (ms / 1e3) / 1e9
    zs = z.float().sum().item()
    out = {
        "metric": "simulated frames/s", "value": J / (ms / 1e3), "unit": "frames/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32 (Poisson draws in f64)",
        "data": "synthetic",
        "config": {"workload": f"simulate {args.config}: object {n}x{n}, probe {np_}x{np_}, {J} positions, "
                               f"Poisson peak {peak:g}"},
        "roofline": {"bound": "hbm", "kernel": "pmace_simulate: frames_k, fft2 passes, intensity_k, poisson_k",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": None, "algorithmic_bytes_per_step": B},
        "wall_s": wall, "photon_scale": scale, "mean_count": zs / z.numel(),
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = simulate_cpu_baseline(x, d, pos, peak, 7)
    print(json.dumps(out), flush=True)


def bench_serve(args):
    print(json.dumps(serve_comparison(args)), flush=True)


def serve_comparison(args):
    """Poisson arrivals of requests drawn from the mixed-size pool: the
    continuous-batching server against the plain FIFO solver."""
    import torch
    from paper_2111_14240_amd import serve
    pool = _mix_problems(args.pool)
    torch.cuda.synchronize()
    rng = np.random.default_rng(5)
    pick = rng.integers(0, len(pool), size=args.requests)
    arrivals = serve.poisson_arrivals(args.requests, args.rate, seed=5)
    rule = _stop_rule(args)
    results = {}
    variants = [(int(v), int(a)) for v in str(args.max_large).split(",")
                for a in str(args.max_active).split(",")]
    names = [(f"served_max_large{v}" if v > 0 else "served_one_class") + f"_active{a}"
             for v, a in variants]
    for name in names + ["plain"]:
        reqs = [serve.Request(i, pool[pick[i]], float(arrivals[i])) for i in range(args.requests)]
        v_split = variants[names.index(name)][0] if name != "plain" else 0
        ex = serve.GPUExecutor(alpha=0.5, split_work=args.large_work if v_split > 0 else None, **rule)
        retire, done_count = ex.retire, [0]

        def retire_and_report(rid, _retire=retire, _name=name):
            done_count[0] += 1
            if done_count[0] % 250 == 0:
                print(f"[serve] {_name}: {done_count[0]} completed", file=sys.stderr, flush=True)
            return _retire(rid)

        ex.retire = retire_and_report
        clock = serve.WallClock()
        if name != "plain":
            v, a = variants[names.index(name)]
            st = serve.Server(ex, capacity_bytes=int(args.capacity_gb * 2**30),
                              max_active=a, iters_per_step=10,
                              large_work=args.large_work if v > 0 else None,
                              max_large=max(v, 1), hold_small=args.hold_small).run(reqs, clock)
        else:
            st = serve.run_plain(ex, reqs, clock, iters_per_step=10)
        torch.cuda.synchronize()
        results[name] = st.as_dict()
        results[name]["median_iterations"] = float(np.median([r.iters for r in reqs]))
        tail = sorted(reqs, key=lambda r: -r.latency)[:max(1, len(reqs) // 100)]
        results[name]["slowest"] = [
            {"latency": round(r.latency, 4), "wait": round(r.admitted - r.arrival, 4),
             "iters": r.iters, "shape": [r.problem.n1, r.problem.np_, r.problem.num_pos]} for r in tail]
        print(f"[serve] {name}: {results[name]}", file=sys.stderr, flush=True)
    out = {
        "metric": "served p50/p99 latency and solves/s vs plain",
        "value": results[names[0]]["solves_per_s"], "unit": "solves/s", "n_gpus": 1,
        "higher_is_better": True, "vs_baseline": None, "dtype": "c64",
        "data": "synthetic (simulated on device)",
        "config": {"workload": f"{args.requests} requests, Poisson arrivals at {args.rate}/s, drawn from "
                               f"{len(pool)} mixed-size problems", "stop_rule": rule,
                   "capacity_GiB": args.capacity_gb, "max_active": args.max_active,
                   "large_work": args.large_work, "policy": names[0]},
        "served": results[names[0]], "plain": results["plain"],
        "served_variants": {n: results[n] for n in names},
    }
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--config", default="c3", choices=["c1", "c2", "c3"])
    ap.add_argument("--method", default="pmace", choices=["pmace", "sharp"],
                    help="plain mode: PMACE (Alg. 1) or SHARP+ (Alg. 2) on the same workload")
    ap.add_argument("--beta", type=float, default=0.8, help="SHARP+ relaxation (the paper grid-searches it)")
    ap.add_argument("--np", type=int, default=0,
                    help="plain mode: probe side other than the config's (same object, raster and step)")
    ap.add_argument("--chunk", type=int, default=0, help="Np > 128: at most this many positions per staging chunk (0 = tuned default)")
    ap.add_argument("--ppw", type=int, default=0,
                    help="plain mode, Np <= 64: patches per workgroup of the whole-patch agent (0 = tuned default)")
    ap.add_argument("--n2", type=int, default=0,
                    help="plain mode: a rectangular object with this many columns (the raster widened "
                         "at the same step)")
    ap.add_argument("--agent", default="default", choices=["default", "staged", "split", "rowspec"],
                    help="plain mode: the library's choice, the three-pass agent (Np > 128), the "
                         "coset-block agent (Np 128/192/256) or the row-spectrum agent (Np > 128)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--systems", action=argparse.BooleanOptionalAction, default=True,
                    help="plain mode: also run the 64-item batch and a short served run against the plain "
                         "solver and add them to the line (--no-systems to skip)")
    ap.add_argument("--serve-requests", type=int, default=600,
                    help="plain mode with --systems: requests in the short served run")
    ap.add_argument("--serve-rate", type=float, default=26.0,
                    help="plain mode with --systems: arrivals per second in the short served run")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="after the run, copy this many MiB three times (counter calibration)")
    ap.add_argument("--mode", default="plain", choices=["plain", "batch", "serve", "simulate"])
    ap.add_argument("--items", type=int, default=64, help="batch mode: reconstructions")
    ap.add_argument("--requests", type=int, default=2000, help="serve mode: requests")
    ap.add_argument("--rate", type=float, default=20.0, help="serve mode: arrivals per second")
    ap.add_argument("--pool", type=int, default=64, help="serve mode: distinct problems")
    ap.add_argument("--capacity-gb", type=float, default=200.0, help="serve mode: workspace budget")
    ap.add_argument("--max-active", default="64",
                    help="serve mode: concurrent requests (comma list of variants)")
    ap.add_argument("--large-work", type=float, default=float(1 << 22),
                    help="serve mode: patch pixels per iteration from which a request is large")
    ap.add_argument("--hold-small", action="store_true",
                    help="serve mode: no small admissions while a large request waits")
    ap.add_argument("--max-large", default="1",
                    help="serve mode: large requests active at once (comma list of variants; 0 = one class)")
    ap.add_argument("--stop", default="nrmse", choices=["nrmse", "data_fit"],
                    help="batch/serve stop rule: NRMSE change (eq. 17) or data-fit cost change (eq. 4)")
    ap.add_argument("--fit-tol", type=float, default=1e-3, help="relative data-fit change for --stop data_fit")
    ap.add_argument("--check-every", type=int, default=1, help="iterations between stop-rule evaluations")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    if args.mode == "batch":
        return bench_batch(args)
    if args.mode == "serve":
        return bench_serve(args)
    if args.mode == "simulate":
        return bench_simulate(args)

    import torch
    from paper_2111_14240_amd import pmace, synth

    cfg = dict(synth.CONFIGS[args.config])
    if args.np:
        cfg["np_"] = args.np
    cfg["scan2"] = cfg["scan"]
    if args.n2:
        # a rectangular object: the config's rows, N2 columns covered by the
        # same step (scan x scan2 raster)
        cfg["scan2"] = (args.n2 - cfg["np_"]) // cfg["step"] + 1
        prob = synth.make_problem(cfg["n"], cfg["np_"], cfg["scan"], cfg["step"], cfg["peak"], cfg["seed"],
                                  name=f"{args.config}-n2{args.n2}", n2=args.n2, scan2=cfg["scan2"])
    elif args.np:
        prob = synth.make_problem(cfg["n"], cfg["np_"], cfg["scan"], cfg["step"], cfg["peak"], cfg["seed"],
                                  name=f"{args.config}-np{args.np}")
    else:
        prob = synth.make_config_problem(args.config)
    alpha, kappa, rho = ALPHA[args.config], synth.KAPPA, synth.RHO
    sharp = args.method == "sharp"
    mkw = dict(method=pmace.PMACE_METHOD_SHARP_PLUS, beta=args.beta) if sharp else {}
    mkw["flags"] = {"default": 0, "staged": pmace.PMACE_STAGED_AGENT, "split": pmace.PMACE_SPLIT_AGENT,
                    "rowspec": pmace.PMACE_ROWSPEC_AGENT}[args.agent]
    mkw["ppw"] = args.ppw
    key = workload_key(args.config, args.method, args.np, args.agent) + (f"-n2{args.n2}" if args.n2 else "")
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(device=dev)
    with torch.cuda.stream(stream):
        R = pmace.Reconstruction(prob.n1, prob.n2, prob.probe, prob.pos, prob.z, alpha, kappa, rho,
                                 device=dev, stream=stream, chunk=args.chunk, **mkw)
        R.iterate(args.warmup)
        R.sync()
        torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        ev0.record(stream)
        R.iterate(args.steps)
        ev1.record(stream)
        R.sync()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        gpu_ms = ev0.elapsed_time(ev1)
        xh = R.reconstruct().cpu().numpy()
        agent = R.agent
    ms_per_step = gpu_ms / args.steps
    J, np_ = prob.num_pos, prob.np_
    value = J * args.steps / (gpu_ms / 1e3)
    B = algorithmic_bytes(J, np_, prob.n1, prob.n2)
    Fl = algorithmic_flops(J, np_)
    achieved = B / (ms_per_step / 1e3) / 1e9
    # NRMSE of the reconstruction after warmup+steps iterations (eq. (17))
    mask = synth.roi_mask(prob.probe, prob.pos, prob.n1, prob.n2)
    a, b = xh[mask].astype(np.complex128), prob.x_true[mask]
    c = np.vdot(b, a)
    nrmse = float(np.linalg.norm(a - np.exp(1j * np.angle(c)) * b) / np.linalg.norm(b))

    out = {
        "metric": ("SHARP+" if sharp else "PMACE") + " patch-updates/s",
        "value": value,
        "unit": "patch-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64",
        "data": "synthetic",
        "config": {"workload": f"{key}: object {prob.n1}x{prob.n2}, probe {np_}x{np_}, "
                               f"{J} positions ({cfg['scan']}x{cfg['scan2']} raster, step {cfg['step']} px"
                               f"{raster_overhang(prob.n1, np_, cfg['scan'], cfg['step'])}), "
                               f"Poisson peak {cfg['peak']}",
                   "method": "SHARP+ (Alg. 2)" if sharp else "PMACE (Alg. 1)",
                   **({"beta": args.beta} if sharp else {"alpha": alpha, "kappa": kappa, "rho": rho}),
                   "chunk": args.chunk,
                   **({"ppw": args.ppw} if args.ppw else {}),
                   "agent": agent,
                   "iteration_graph": "HIP graphs of 32 iterations (single-iteration graph for the rest)"},
        "roofline": {"bound": "hbm", "kernel": iteration_kernels(np_, J, args.method, agent),
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(key),
                     "traffic_level": TRAFFIC_LEVEL, "algorithmic_bytes_per_step": B},
        "alu": {"algorithmic_flops_per_step": Fl,
                "achieved_tflops": Fl / (ms_per_step / 1e3) / 1e12,
                "peak_tflops": FP32_VECTOR_PEAK_TFLOPS},
        "wall_s": wall,
        "nrmse_after_run": nrmse,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(prob, alpha, kappa, rho, method=args.method, beta=args.beta)
        out["cpu_baseline_all_cores"] = cpu_baseline_all_cores(prob, alpha, kappa, rho, method=args.method,
                                                               beta=args.beta)
    if args.copy_mib:
        calibration_copy(args.copy_mib)
    if args.systems:
        # the metric's second half: the mixed-size batch (64 reconstructions)
        # and a short served run, each against the plain one-at-a-time solver
        # on this GPU, to the same on-device stop rule
        del R
        torch.cuda.empty_cache()
        b = batch_comparison(args)
        out["batched_vs_plain"] = {k: b[k] for k in ("batched", "plain", "speedup", "same_iterations",
                                                     "same_nrmse", "iterations", "nrmse")}
        out["batched_vs_plain"]["workload"] = b["config"]["workload"]
        sargs = argparse.Namespace(**vars(args))
        sargs.requests = args.serve_requests
        sargs.rate = args.serve_rate
        sv = serve_comparison(sargs)
        keep = ("solves_per_s", "p50", "p99", "mean_latency", "completed", "max_active")
        out["served_vs_plain"] = {"workload": sv["config"]["workload"], "policy": sv["config"]["policy"],
                                  "served": {k: sv["served"].get(k) for k in keep},
                                  "plain": {k: sv["plain"].get(k) for k in keep}}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
