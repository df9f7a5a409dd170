"""The launch-shape tuner's choice logic on synthetic timings (CPU): each
family is decided by the workloads it was timed on, and the row/column block
search, timed on Np = 256, sets the 256-point row block only."""
from paper_2111_14240_amd import tune


def _times(cands, **override):
    t = {n: {"np128": 1.0, "np256": 1.0, "np32": 1.0, "np48": 1.0, "np64": 1.0} for n in cands}
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


def test_patches_per_workgroup_per_side():
    res = {"np32_ppw1": 1.0, "np32_ppw2": 0.95, "np32_ppw4": 0.9, "np32_ppw8": 0.9,
           "np48_ppw1": 1.0, "np48_ppw2": 1.0, "np48_ppw4": 1.1, "np64_ppw1": 0.8, "np64_ppw2": 0.9}
    # ties keep the smaller value
    assert tune._pick_ppw(res) == {"PMACE_PPW32": 4, "PMACE_PPW48": 1, "PMACE_PPW64": 1}


def test_ppw_choices_fit_a_workgroup():
    # every value timed keeps ppw x Np x (threads per line) <= 1024 with the tuned line splits
    d = dict(tune.DEFAULTS)
    import json, os
    if os.path.exists(tune.TUNED):
        d.update(json.load(open(tune.TUNED))["defines"])
    for n, ks in tune.PPW_SPACE.items():
        a = {32: d["PMACE_GEO32_A"], 48: 4, 64: d["PMACE_GEO64_A"]}[n]
        assert max(ks) * n * a <= 1024, n


def test_agent_sides_bitmasks():
    res = {"np128_other": 1.0, "np128_split": 1.2, "np160_other": 1.0, "np160_rowspec": 1.1,
           "np192_other": 1.0, "np192_split": 0.9, "np192_rowspec": 0.95,
           "np256_other": 1.0, "np256_split": 1.1, "np256_rowspec": 1.2}
    assert tune._agent_sides(res) == (2, 0)
    res["np128_split"] = 0.5
    res["np256_split"] = 0.5
    assert tune._agent_sides(res) == (7, 0)
    # the row-spectrum agent wins 160 and 256; 192 stays split
    res.update({"np160_rowspec": 0.8, "np256_rowspec": 0.4})
    assert tune._agent_sides(res) == (3, 5)
    # every side's candidates are timed and map to a bit of their mask
    for np_, (wl, names) in tune.AGENT_SIDES.items():
        assert wl in tune.WORKLOADS and tune.WORKLOADS[wl][1] == np_
        assert all(np_ in tune.SPLIT_BIT for n in names if n == "split")
        assert all(np_ in tune.ROWSPEC_BIT for n in names if n == "rowspec")


def test_line_split_of_128_points():
    cands = tune.candidates()
    assert "geo128a4" in cands and cands["geo128a4"]["PMACE_GEO128_A"] == 4
    d, _, _ = tune._pick(cands, _times(cands, geo128a4=("np128", 0.9)))
    assert d["PMACE_GEO128_A"] == 4
    d, _, _ = tune._pick(cands, _times(cands, geo128a4=("np128", 1.1)))
    assert d["PMACE_GEO128_A"] == 8


def test_row_consensus_width():
    cands = tune.candidates()
    # every width is built with Np = 256 on the row-spectrum agent
    for t in tune.CRT_SPACE:
        assert cands[f"crt{t}"]["PMACE_CR_T"] == t and cands[f"crt{t}"]["PMACE_ROWSPEC_SIDES"] == 4
    d, _, _ = tune._pick(cands, _times(cands, crt512=("np256", 0.9)))
    assert d["PMACE_CR_T"] == 512
    # a tie keeps the smaller width; the pick never sets the agent sides
    d, _, _ = tune._pick(cands, _times(cands))
    assert d["PMACE_CR_T"] == 256 and "PMACE_ROWSPEC_SIDES" not in d


def test_chunk_bounds_per_agent():
    res = {f"np256_chunk{c}": 1.0 for c in tune.CHUNKS_RS}
    assert tune._best_chunk(res, tune.CHUNKS_RS) == min(tune.CHUNKS_RS)   # ties keep the smaller
    res["np256_chunk1600"] = 0.9
    assert tune._best_chunk(res, tune.CHUNKS_RS) == 1600


def test_sharp_plus_agent_choice():
    assert tune._sharp_rowspec({"sharp_np256_other": 1.6, "sharp_np256_rowspec": 1.36}) == 1
    assert tune._sharp_rowspec({"sharp_np256_other": 1.3, "sharp_np256_rowspec": 1.36}) == 0
