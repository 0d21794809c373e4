"""The autotuner: searches tile slots x tile height on the job, keeps only
candidates within the accuracy budget, caches and logs its choice."""

import json
import math

import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def test_autotune_selfjoin_and_cache(tmp_path, monkeypatch):
    import paper_1904_12626_amd as mpx
    from paper_1904_12626_amd import autotune as AT
    cache = tmp_path / "autotune.json"
    monkeypatch.setenv("MPX_AUTOTUNE_CACHE", str(cache))
    T = torch.from_numpy(W.random_walk(40000, 11)).to(DEV)
    m, ez = 128, 32
    lines = []
    choice = AT.tune_selfjoin(T, m, ez, log=lines.append)
    assert choice["tile_slots"] in AT.SLOTS and choice["reseed_rows"] in AT.ROWS
    rec = json.loads(cache.read_text())
    (key, entry), = rec.items()
    assert entry["choice"] == choice
    trials = entry["trials"]
    assert len(trials) == len(AT.SLOTS) * len(AT.ROWS)
    budget = entry["budget"]
    assert math.isclose(budget, 0.5 * 1e-3 * math.sqrt(m))
    ok = [t for t in trials if t.get("within_budget")]
    assert ok, "no candidate within the budget"
    best = min(ok, key=lambda t: t["sweep_ms"])
    assert (best["tile_slots"], best["reseed_rows"]) == (choice["tile_slots"], choice["reseed_rows"])
    for t in trials:
        if "raw_max_abs_dP_vs_f64" in t:
            assert t["within_budget"] == (t["raw_max_abs_dP_vs_f64"] <= budget
                                          and t["index_excess_vs_f64"] <= budget)
    assert entry["space"] == {"tile_slots": list(AT.SLOTS), "reseed_rows": list(AT.ROWS)}
    assert any("chose" in s for s in lines)
    # a second call answers from the cache, and the chosen options reproduce
    # a profile within the budget of the FP64 sweep
    again = AT.tune_selfjoin(T, m, ez, log=lines.append)
    assert again == choice
    P, _ = mpx.selfjoin(T, m, ez, tile_slots=choice["tile_slots"], reseed_rows=choice["reseed_rows"],
                        fp64_finalize=False)
    P64, _ = mpx.selfjoin(T, m, ez, precision="f64")
    assert float((P.double() - P64.double()).abs().max()) <= budget
