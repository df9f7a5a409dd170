"""The launch-shape tuner's choice logic on synthetic timings (CPU): each
family is decided by the workloads it was timed on, and the row/column block
search, timed on Np = 256, sets the 256-point row block only."""
from paper_2111_14240_amd import tune


def _times(cands, **override):
    t = {n: {"np128": 1.0, "np256": 1.0, "np32": 1.0, "np64": 1.0} for n in cands}
    for name, (wl, v) in override.items():
        t[name][wl] = v
    return t


def test_defaults_when_nothing_is_faster():
    cands = tune.candidates()
    d, _, _ = tune._pick(cands, _times(cands))
    assert d == tune.DEFAULTS


def test_block_search_sets_the_256_row_block_only():
    cands = tune.candidates()
    d, _, b = tune._pick(cands, _times(cands, rb8cb32=("np256", 0.9)))
    assert d["PMACE_RB256"] == 8 and d["PMACE_CB"] == 32
    assert d["PMACE_RB"] == tune.DEFAULTS["PMACE_RB"]
    assert min(b, key=b.get) == "rb8cb32"


def test_gather_and_split_choices():
    cands = tune.candidates()
    t = _times(cands, g2u8c32=("np128", 0.8), geo32a2=("np32", 0.9))
    t["g2u8c32"]["np256"] = 0.95
    d, score, _ = tune._pick(cands, t)
    assert (d["PMACE_GT_K"], d["PMACE_GATHER_UNROLL"], d["PMACE_GT_C"]) == (2, 8, 32)
    assert d["PMACE_GEO32_A"] == 2 and d["PMACE_GEO64_A"] == tune.DEFAULTS["PMACE_GEO64_A"]
