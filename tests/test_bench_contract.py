"""bench.py's output contract: one JSON line with the metric, the roofline
object and the CPU baseline (GPU), and a clear refusal of more than one GPU
(CPU: the refusal comes before anything touches a device)."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(args, timeout=300):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True,
                          text=True, timeout=timeout, cwd=ROOT)


def test_more_than_one_gpu_is_refused():
    r = _run(["--gpus", "2"], timeout=120)
    assert r.returncode == 2
    out = json.loads(r.stdout.strip().splitlines()[-1])
    assert out["n_gpus"] == 2 and "one GPU" in out["error"]


@pytest.mark.gpu
def test_bench_line_has_the_contract_fields():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    print("[bench-contract] c1, 5 steps, small systems legs", flush=True)
    r = _run(["--config", "c1", "--steps", "5", "--warmup", "1", "--items", "6", "--pool", "6",
              "--serve-requests", "12"])
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [ln for ln in r.stdout.splitlines() if ln.startswith("{")]
    assert len(lines) == 1
    d = json.loads(lines[0])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
              "scaling", "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert k in d, k
    assert d["n_gpus"] == 1 and d["steps"] == 5 and d["warmup"] == 1 and d["value"] > 0
    assert "workload" in d["config"]
    rl = d["roofline"]
    assert rl["bound"] == "hbm" and rl["unit"] == "GB/s" and rl["peak"] == 8000.0
    assert abs(rl["frac"] - rl["achieved"] / rl["peak"]) < 1e-12
    assert "traffic" in rl
    cb = d["cpu_baseline"]
    assert cb["kind"] == "oracle" and cb["cores"] >= 1 and cb["value"] > 0 and cb["sample"]
    assert cb["cpu_model"] and cb["host_cpu_count"] >= 1
    ca = d["cpu_baseline_all_cores"]
    assert ca["kind"] == "oracle" and ca["cores"] >= 1 and ca["value"] > 0
    bp = d["batched_vs_plain"]
    assert bp["batched"]["solves_per_s"] > 0 and bp["plain"]["solves_per_s"] > 0 and bp["same_iterations"]
    sp = d["served_vs_plain"]
    assert sp["served"]["completed"] == 12 and sp["plain"]["completed"] == 12
    assert sp["served"]["p99"] >= sp["served"]["p50"] > 0


@pytest.mark.gpu
@pytest.mark.parametrize("args,metric", [
    (["--config", "c1", "--method", "sharp", "--steps", "4", "--warmup", "1", "--no-systems"],
     "SHARP+ patch-updates/s"),
    (["--config", "c1", "--np", "48", "--steps", "4", "--warmup", "1", "--no-systems"], "PMACE patch-updates/s"),
    (["--mode", "simulate", "--config", "c1", "--steps", "3", "--warmup", "1"], "simulated frames/s"),
])
def test_variant_lines(args, metric):
    """SHARP+, another probe side and the simulator print the same kind of
    line, each with its roofline and the oracle's baseline."""
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    print("[bench-contract]", " ".join(args), flush=True)
    r = _run(args)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [ln for ln in r.stdout.splitlines() if ln.startswith("{")]
    assert len(lines) == 1
    d = json.loads(lines[0])
    assert d["metric"] == metric and d["value"] > 0 and d["n_gpus"] == 1
    rl = d["roofline"]
    assert rl["bound"] == "hbm" and abs(rl["frac"] - rl["achieved"] / rl["peak"]) < 1e-12
    assert d["cpu_baseline"]["kind"] == "oracle" and d["cpu_baseline"]["value"] > 0
    if "--np" in args:
        assert "probe 48x48" in d["config"]["workload"]


def test_traffic_table_lookup(tmp_path, monkeypatch):
    """bench.py reports the counter-measured traffic only for the kernel
    sources it was measured on: the table row's hash must equal the hash of
    the current sources, otherwise `traffic` is null."""
    import importlib.util
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    h = bench.kernel_source_hash()
    assert len(h) == 16 and int(h, 16) >= 0
    assert bench.workload_key("c3", "pmace", 0) == "c3"
    assert bench.workload_key("c3", "sharp", 0) == "c3-sharp"
    assert bench.workload_key("c3", "pmace", 192, "staged") == "c3-np192-staged"
    table = tmp_path / "traffic.md"
    table.write_text("| workload | kernel sources | a | b | c | d | bytes |\n"
                     f"| c3 | {h} | 1 | 2 | 3 | 4 | 6.5e+09 |\n"
                     "| c2 | 0000000000000000 | 1 | 2 | 3 | 4 | 1.0e+08 |\n")
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(table))
    assert bench.measured_traffic("c3") == 6.5e9
    assert bench.measured_traffic("c2") is None          # measured on other sources
    assert bench.measured_traffic("c1") is None          # not measured
