"""Autotuner for the launch shapes of the PMACE kernels.

The tunables are compile-time parameters of libpmace.so (see
csrc/pmace_internal.hpp) plus one run-time default:

    PMACE_GT_K           threads per object pixel in the consensus gather (1, 2, 4)
    PMACE_GATHER_UNROLL  loads in flight per gather thread (8, 16)
    PMACE_GT_C           gather tile width in object pixels (32, 64)
    PMACE_RB256          Np = 256 row passes: patch rows per workgroup (8, 16, 32)
    PMACE_RB             Np = 160, 192 row passes: patch rows per workgroup (fixed, 32)
    PMACE_CB             Np > 128 column pass: patch columns per workgroup (16, 32)
    PMACE_CHUNK256       Np > 128, three-pass agent: positions per chunk (stage buffer size)
    PMACE_CHUNK256_RS    the same for the row-spectrum agent
    PMACE_GEO32_A        32-point line split over threads: 4 x 8 or 2 x 16 registers
    PMACE_GEO64_A        64-point line split: 8 x 8 or 4 x 16
    PMACE_GEO128_A       128-point line split: 8 x 16 or 4 x 32
    PMACE_CR_T           row-spectrum consensus: threads per workgroup (256, 512, 1024)
    PMACE_PPW32/48/64    (run-time choice, recorded as the build's default) patches per
                         workgroup of the whole-patch agent for Np = 32, 48, 64
    PMACE_SPLIT_SIDES    (run-time choice, recorded for the build) which of Np = 128, 192, 256
                         default to the split (coset-block) agent: bit 0, 1, 2
    PMACE_ROWSPEC_SIDES  (likewise) which of Np = 160, 192, 256 default to the row-spectrum
                         agent: bit 0, 1, 2
    PMACE_ROWSPEC_SHARP  (likewise) 1: SHARP+ takes the row-spectrum agent on those sides too

Search (coordinate-wise, every candidate measured on the device):
  1. gather shape (GT_K x unroll x tile width) with the default row/column blocks, scored by
     the iteration time of a Np = 128 and a Np = 256 workload;
  2. row/column blocks with the default gather, scored on the Np = 256 workload
     (the row block found applies to 256-point lines; 160 and 192 keep PMACE_RB);
  3. the line-FFT split (radix) of Np = 32, 64 and 128, each on a workload of its size,
     and the row-spectrum consensus width on the Np = 256 workload (that agent forced
     for the side);
  4. the chunk size of each large-side agent (three-pass, row-spectrum), at run time,
     with the combined choice;
  5. patches per workgroup of the whole-patch agent (Np = 32, 48, 64), at run
     time, each on a workload of its size, with the built library;
  6. the agent of each side that has several (Np = 128: whole patch or split;
     160: three-pass or row-spectrum; 192 and 256: three-pass, split or
     row-spectrum), at run time, with the built library.
Each candidate library is built into a scratch directory and timed in a
process of its own.  The choice is written to tuned.json beside this file;
build.py passes it to hipcc as -D flags.

    python -m paper_2111_14240_amd.tune build DIR      # compile candidates (no GPU)
    python -m paper_2111_14240_amd.tune time DIR       # time them (GPU), write DIR/times.json
    python -m paper_2111_14240_amd.tune pick DIR       # write tuned.json from the times
    python -m paper_2111_14240_amd.tune chunk          # time chunk sizes with the built library
    python -m paper_2111_14240_amd.tune ppw            # time patches per workgroup (built library)
    python -m paper_2111_14240_amd.tune agent          # time the agents of each side (built library)
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import json
import os
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
TUNED = os.path.join(HERE, "tuned.json")
DEFAULTS = {"PMACE_GT_K": 1, "PMACE_GATHER_UNROLL": 8, "PMACE_GT_C": 64, "PMACE_RB": 32, "PMACE_RB256": 16,
            "PMACE_CB": 16, "PMACE_GEO32_A": 4, "PMACE_GEO64_A": 8, "PMACE_GEO128_A": 8,
            "PMACE_PPW32": 1, "PMACE_PPW48": 1, "PMACE_PPW64": 1, "PMACE_CR_T": 256}
GATHER_SPACE = [(k, u, c) for k in (1, 2, 4) for u in (8, 16) for c in (64, 32)]
BLOCK_SPACE = [(rb, cb) for rb in (8, 16, 32) for cb in (16, 32)]
GEO_SPACE = [(32, 2), (64, 4), (128, 4)]   # the non-default splits
CRT_SPACE = (256, 512, 1024)                # row-spectrum consensus threads per workgroup
PPW_SPACE = {32: (1, 2, 4, 8), 48: (1, 2, 4), 64: (1, 2)}   # patches per workgroup per side
# Agents timed per side ("other": the whole-patch agent for 128, three-pass above).
AGENT_SIDES = {128: ("np128", ("other", "split")), 160: ("np160", ("other", "rowspec")),
               192: ("np192", ("other", "split", "rowspec")), 256: ("np256", ("other", "split", "rowspec"))}
CHUNKS = (64, 128, 192, 256, 400)            # three-pass agent (PMACE_CHUNK256)
CHUNKS_RS = (256, 400, 800, 1600, 4096)      # row-spectrum agent (PMACE_CHUNK256_RS)

# Tuning workloads: (object side, probe side, scan side, step, peak photons).
WORKLOADS = {"np128": (512, 128, 15, 24, 1e5), "np256": (1024, 256, 40, 20, 1e6),
             "np32": (256, 32, 14, 16, 1e5), "np64": (512, 64, 20, 22, 1e5),
             "np48": (384, 48, 20, 16, 1e5), "np192": (1024, 192, 40, 20, 1e6),
             "np160": (1024, 160, 40, 20, 1e6)}


def candidates():
    """Name -> defines of every candidate library."""
    out = {}
    for k, u, c in GATHER_SPACE:
        d = dict(DEFAULTS, PMACE_GT_K=k, PMACE_GATHER_UNROLL=u, PMACE_GT_C=c)
        out[f"g{k}u{u}" + ("" if c == 64 else f"c{c}")] = d
    for rb, cb in BLOCK_SPACE:
        d = dict(DEFAULTS, PMACE_RB256=rb, PMACE_CB=cb)
        out[f"rb{rb}cb{cb}"] = d
    for n, a in GEO_SPACE:
        d = dict(DEFAULTS, **{f"PMACE_GEO{n}_A": a})
        out[f"geo{n}a{a}"] = d
    for t in CRT_SPACE:     # Np = 256 on the row-spectrum agent in these builds
        out[f"crt{t}"] = dict(DEFAULTS, PMACE_CR_T=t, PMACE_ROWSPEC_SIDES=4)
    # the default appears in both families: keep one copy
    uniq, seen = {}, set()
    for name, d in out.items():
        key = tuple(sorted(d.items()))
        if key not in seen:
            seen.add(key)
            uniq[name] = d
    return uniq


def cmd_build(args):
    from . import build as B
    os.makedirs(args.dir, exist_ok=True)
    cands = candidates()
    if args.family:
        cands = {n: d for n, d in cands.items() if n.startswith(args.family) or n == "g1u8"}
    with open(os.path.join(args.dir, "candidates.json"), "w") as f:
        json.dump(cands, f, indent=1)

    def one(item):
        name, d = item
        lib = os.path.join(args.dir, f"libpmace_{name}.so")
        B.build(out=lib, defines=d)
        return name

    with cf.ThreadPoolExecutor(max_workers=args.jobs) as ex:
        for name in ex.map(one, sorted(cands.items())):
            print("built", name, flush=True)


def _time_library(lib, workloads, iters, chunks=(0,), flags=0, ppw=0, method=0):
    """Run in a fresh process: load `lib`, time `iters` iterations (one graph
    replay each) per workload, return ms per iteration (method 1: SHARP+,
    beta 0.8)."""
    import torch
    from . import pmace
    pmace.load_library(lib)
    res = {}
    for wl in workloads:
        n, np_, scan, step, peak = WORKLOADS[wl]
        prob = pmace.simulated_problem(n, np_, scan, step, peak, seed=7)
        for ch in chunks:
            stream = torch.cuda.Stream()
            with torch.cuda.stream(stream):
                R = pmace.Reconstruction(n, n, prob.probe, prob.pos, prob.z, 0.5, chunk=ch,
                                         stream=stream, flags=flags, ppw=ppw, method=method,
                                         beta=0.8 if method else 0.5)
                R.iterate(3)
                R.sync()
                best = float("inf")
                for _ in range(3):
                    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    e0.record(stream)
                    R.iterate(iters)
                    e1.record(stream)
                    R.sync()
                    best = min(best, e0.elapsed_time(e1) / iters)
                R.close()
            res[wl if ch == 0 else f"{wl}_chunk{ch}"] = best
            print(f"  {os.path.basename(lib)} {wl} chunk {ch}: {best:.4f} ms/iteration", flush=True)
    return res


def cmd_time(args):
    cands = json.load(open(os.path.join(args.dir, "candidates.json")))
    times = {}
    for name in sorted(cands):
        lib = os.path.join(args.dir, f"libpmace_{name}.so")
        if name == "g1u8":       # the default build is also timed on the small sizes
            wl_extra = ["np32", "np48", "np64"]
        else:
            wl_extra = []
        if name.startswith("geo128"):
            wl = ["np128"]
        elif name.startswith("geo"):
            wl = ["np32", "np64"]

        elif name.startswith("g"):
            wl = ["np128", "np256"]
        else:
            wl = ["np256"]
        out = subprocess.run([sys.executable, "-m", "paper_2111_14240_amd.tune", "_one", lib,
                              ",".join(wl + wl_extra), str(args.iters)],
                             capture_output=True, text=True, timeout=300,
                             cwd=os.path.dirname(HERE))
        sys.stdout.write(out.stdout)
        if out.returncode != 0:
            sys.stderr.write(out.stderr[-2000:])
            raise SystemExit(f"timing {name} failed with status {out.returncode}")
        times[name] = json.loads(out.stdout.strip().splitlines()[-1])
    with open(os.path.join(args.dir, "times.json"), "w") as f:
        json.dump(times, f, indent=1)


def cmd_one(args):
    res = _time_library(args.lib, args.workloads.split(","), args.iters)
    print(json.dumps(res), flush=True)


def _pick(cands, times):
    import math
    g = {n: t for n, t in times.items() if n.startswith("g") and not n.startswith("geo")}
    base = g["g1u8"]
    # geometric mean of the speedups over the default on both workloads
    score = {n: math.sqrt((base["np128"] / t["np128"]) * (base["np256"] / t["np256"])) for n, t in g.items()}
    best_g = max(score, key=score.get)
    # the default first, so that a tie keeps it
    b = {"rb16cb16": base["np256"]}
    b.update({n: t["np256"] for n, t in times.items() if n.startswith("rb")})
    best_b = min(b, key=b.get)
    d = dict(DEFAULTS)
    d["PMACE_GT_K"] = cands[best_g]["PMACE_GT_K"]
    d["PMACE_GATHER_UNROLL"] = cands[best_g]["PMACE_GATHER_UNROLL"]
    d["PMACE_GT_C"] = cands[best_g].get("PMACE_GT_C", 64)
    rb, cb = best_b[2:].split("cb")
    d["PMACE_RB256"], d["PMACE_CB"] = int(rb), int(cb)
    # line splits: the default build's time on each size against the variant's
    for n, a in GEO_SPACE:
        key, wl = f"geo{n}a{a}", f"np{n}"
        if key in times and wl in base and times[key][wl] < base[wl]:
            d[f"PMACE_GEO{n}_A"] = a
    # row-spectrum consensus width (ties keep the smaller)
    crt = {t: times[f"crt{t}"]["np256"] for t in CRT_SPACE if f"crt{t}" in times}
    if crt:
        d["PMACE_CR_T"] = min(sorted(crt), key=crt.get)
    return d, score, b


def cmd_pick(args):
    cands = json.load(open(os.path.join(args.dir, "candidates.json")))
    times = json.load(open(os.path.join(args.dir, "times.json")))
    rec = {}
    if os.path.exists(TUNED):
        rec = json.load(open(TUNED))
    d, score, b = _pick(cands, times)
    rec["defines"] = dict(rec.get("defines", {}), **d)
    rec["gather_scores"] = score
    rec["block_ms_np256"] = b
    rec["times_ms"] = times
    rec["when"] = time.strftime("%Y-%m-%d %H:%M")
    with open(TUNED, "w") as f:
        json.dump(rec, f, indent=1, sort_keys=True)
    print(json.dumps(rec["defines"]))


def _best_chunk(res, chunks):
    """The chunk bound with the least time (ties keep the smaller)."""
    return min(chunks, key=lambda c: res[f"np256_chunk{c}"])


def cmd_chunk(args):
    """Chunk bounds at Np = 256 with the built library: the three-pass agent's
    (PMACE_CHUNK256) and the row-spectrum agent's (PMACE_CHUNK256_RS), each
    with that agent forced."""
    from . import build as B
    from . import pmace
    res = _time_library(B.LIB, ["np256"], args.iters, chunks=CHUNKS, flags=pmace.PMACE_STAGED_AGENT)
    res_rs = _time_library(B.LIB, ["np256"], args.iters, chunks=CHUNKS_RS, flags=pmace.PMACE_ROWSPEC_AGENT)
    best, best_rs = _best_chunk(res, CHUNKS), _best_chunk(res_rs, CHUNKS_RS)
    rec = json.load(open(TUNED)) if os.path.exists(TUNED) else {"defines": dict(DEFAULTS)}
    rec["chunk_ms_np256"] = res
    rec["chunk_ms_np256_rowspec"] = res_rs
    if args.write:
        rec["defines"]["PMACE_CHUNK256"] = best
        rec["defines"]["PMACE_CHUNK256_RS"] = best_rs
        with open(TUNED, "w") as f:
            json.dump(rec, f, indent=1, sort_keys=True)
    print(json.dumps({"best_chunk": best, "best_chunk_rowspec": best_rs, **res,
                      **{f"rowspec_{k}": v for k, v in res_rs.items()}}))


def _pick_ppw(res):
    """Per side, the patches per workgroup with the least time (ties keep the
    smaller value)."""
    out = {}
    for n, ks in sorted(PPW_SPACE.items()):
        t = {k: res[f"np{n}_ppw{k}"] for k in ks if f"np{n}_ppw{k}" in res}
        if t:
            out[f"PMACE_PPW{n}"] = min(sorted(t), key=t.get)
    return out


def cmd_ppw(args):
    """Time each patches-per-workgroup choice of the whole-patch agent on a
    workload of each side (alternating, best of `rounds`) with the built
    library, and record the fastest as the build's default for that side."""
    from . import build as B
    res = {}
    for n, ks in sorted(PPW_SPACE.items()):
        wl = f"np{n}"
        for _ in range(args.rounds):
            for k in ks:
                t = _time_library(B.LIB, [wl], args.iters, ppw=k)[wl]
                res[f"{wl}_ppw{k}"] = min(res.get(f"{wl}_ppw{k}", float("inf")), t)
    d = _pick_ppw(res)
    rec = json.load(open(TUNED)) if os.path.exists(TUNED) else {"defines": dict(DEFAULTS)}
    rec["ppw_ms"] = res
    if args.write:
        rec["defines"].update(d)
        with open(TUNED, "w") as f:
            json.dump(rec, f, indent=1, sort_keys=True)
    print(json.dumps({**d, **res}))


SPLIT_BIT = {128: 0, 192: 1, 256: 2}     # PMACE_SPLIT_SIDES
ROWSPEC_BIT = {160: 0, 192: 1, 256: 2}   # PMACE_ROWSPEC_SIDES


def _sharp_rowspec(res):
    """PMACE_ROWSPEC_SHARP: 1 where SHARP+ at Np = 256 ran faster on the
    row-spectrum agent than on the three-pass one."""
    return 1 if res["sharp_np256_rowspec"] < res["sharp_np256_other"] else 0


def _agent_sides(res):
    """(PMACE_SPLIT_SIDES, PMACE_ROWSPEC_SIDES) from the agent times: each side
    defaults to its fastest agent (ties keep the earlier one in AGENT_SIDES)."""
    split = rowspec = 0
    for np_, (wl, names) in sorted(AGENT_SIDES.items()):
        best = min(names, key=lambda n: res[f"{wl}_{n}"])
        if best == "split":
            split |= 1 << SPLIT_BIT[np_]
        elif best == "rowspec":
            rowspec |= 1 << ROWSPEC_BIT[np_]
    return split, rowspec


def cmd_agent(args):
    """Per side with several agents, time each (alternating, best of `rounds`)
    with the built library and record the fastest as that side's default."""
    from . import build as B
    from . import pmace
    flag = {"other": pmace.PMACE_STAGED_AGENT, "split": pmace.PMACE_SPLIT_AGENT,
            "rowspec": pmace.PMACE_ROWSPEC_AGENT}
    res = {}
    for np_, (wl, names) in sorted(AGENT_SIDES.items()):
        for _ in range(args.rounds):
            for name in names:
                t = _time_library(B.LIB, [wl], args.iters, flags=flag[name])[wl]
                res[f"{wl}_{name}"] = min(res.get(f"{wl}_{name}", float("inf")), t)
    for _ in range(args.rounds):       # SHARP+ (no split agent) at Np = 256
        for name in ("other", "rowspec"):
            t = _time_library(B.LIB, ["np256"], args.iters, flags=flag[name], method=1)["np256"]
            res[f"sharp_np256_{name}"] = min(res.get(f"sharp_np256_{name}", float("inf")), t)
    split, rowspec = _agent_sides(res)
    sharp_rs = _sharp_rowspec(res)
    rec = json.load(open(TUNED)) if os.path.exists(TUNED) else {"defines": dict(DEFAULTS)}
    rec["agent_ms"] = res
    if args.write:
        rec["defines"]["PMACE_SPLIT_SIDES"] = split
        rec["defines"]["PMACE_ROWSPEC_SIDES"] = rowspec
        rec["defines"]["PMACE_ROWSPEC_SHARP"] = sharp_rs
        with open(TUNED, "w") as f:
            json.dump(rec, f, indent=1, sort_keys=True)
    print(json.dumps({"PMACE_SPLIT_SIDES": split, "PMACE_ROWSPEC_SIDES": rowspec,
                      "PMACE_ROWSPEC_SHARP": sharp_rs, **res}))


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="cmd", required=True)
    p = sub.add_parser("build")
    p.add_argument("dir")
    p.add_argument("--jobs", type=int, default=4)
    p.add_argument("--family", default="", help="only candidates whose name starts with this (and g1u8)")
    p.set_defaults(fn=cmd_build)
    p = sub.add_parser("time")
    p.add_argument("dir")
    p.add_argument("--iters", type=int, default=20)
    p.set_defaults(fn=cmd_time)
    p = sub.add_parser("_one")
    p.add_argument("lib")
    p.add_argument("workloads")
    p.add_argument("iters", type=int)
    p.set_defaults(fn=cmd_one)
    p = sub.add_parser("pick")
    p.add_argument("dir")
    p.set_defaults(fn=cmd_pick)
    p = sub.add_parser("chunk")
    p.add_argument("--iters", type=int, default=20)
    p.add_argument("--write", action="store_true")
    p.set_defaults(fn=cmd_chunk)
    p = sub.add_parser("ppw")
    p.add_argument("--iters", type=int, default=50)
    p.add_argument("--rounds", type=int, default=3)
    p.add_argument("--write", action="store_true")
    p.set_defaults(fn=cmd_ppw)
    p = sub.add_parser("agent")
    p.add_argument("--iters", type=int, default=20)
    p.add_argument("--rounds", type=int, default=2)
    p.add_argument("--write", action="store_true")
    p.set_defaults(fn=cmd_agent)
    args = ap.parse_args(argv)
    args.fn(args)


if __name__ == "__main__":
    main()
