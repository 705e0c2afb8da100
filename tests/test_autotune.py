"""The autotuner's host logic (paper_2009_06657_amd/autotune.py) on the CPU: the coordinate search
keeps the fastest value of each field when it beats the current choice by more than the noise
margin, skips values the library rejects and the overlap-only fields on one stream; the committed
table holds only fields and values that include/lrdm.h's lrdm_tuning admits."""
import json
import os

import pytest

from paper_2009_06657_amd import autotune


def fake_timer(costs, rejected=()):
    calls = []

    def time_with(t):
        calls.append(dict(t))
        for f, v in t.items():
            if (f, v) in rejected:
                raise ValueError("rejected")
        return 1.0 + sum(costs.get((f, v), 0.0) for f, v in t.items())
    return time_with, calls


def test_search_keeps_the_fastest_value_per_field():
    tw, calls = fake_timer({("gram_blocks", 192): -0.10, ("gram_blocks", 224): -0.05,
                            ("gate_local_max", 6): -0.02, ("gram4_blocks", 128): +0.3})
    best, t_best, t_def, seen = autotune.search(tw, overlap=True)
    assert best == {"gram_blocks": 192, "gate_local_max": 6}
    assert t_def == 1.0 and t_best == pytest.approx(0.88)
    assert calls[0] == {}                                   # the defaults first
    # one field changes at a time: every other candidate of every field is timed once
    assert len(calls) == 1 + sum(len(v) - 1 for v in autotune.CANDIDATES.values())


def test_search_noise_margin_and_rejections():
    tw, _ = fake_timer({("gram_blocks", 128): -0.005, ("aux_cus", 64): -0.2}, rejected={("aux_cus", 64)})
    best, t_best, _, seen = autotune.search(tw, overlap=True)
    assert best == {}                                       # 0.5 % is inside the 1 % noise margin
    assert t_best == 1.0
    assert '{"aux_cus": 64}' not in seen                    # the library rejected it


def test_single_stream_skips_overlap_fields():
    tw, calls = fake_timer({("gram4_blocks", 128): -0.5, ("aux_cus", 64): -0.5})
    best, _, _, _ = autotune.search(tw, overlap=False)
    assert best == {}
    assert not any("gram4_blocks" in c or "aux_cus" in c for c in calls)


def test_key_and_load_roundtrip(tmp_path):
    p = tmp_path / "t.json"
    k = autotune.key(20, 64, "c64", True)
    assert k == "n20_r64_c64_overlap"
    p.write_text(json.dumps({"entries": {k: {"tuning": {"gram_blocks": 192}}}}))
    assert autotune.load(20, 64, "c64", True, str(p)) == {"gram_blocks": 192}
    assert autotune.load(20, 64, "c64", False, str(p)) is None
    assert autotune.load(20, 64, "c64", True, str(tmp_path / "missing.json")) is None


def test_committed_table_is_within_the_abi_ranges():
    if not os.path.exists(autotune.TABLE):
        pytest.skip("no tuning table committed")
    table = json.load(open(autotune.TABLE))
    for k, e in table["entries"].items():
        n, r, dt, mode = k.split("_")
        assert n[0] == "n" and r[0] == "r" and dt in ("c64", "c128") and mode in ("overlap", "single")
        for f, v in e["tuning"].items():
            assert f in autotune.CANDIDATES
            if f == "gram_blocks":
                assert 1 <= v <= 256
            elif f == "gram4_blocks":
                assert 2 <= v <= 256 and mode == "overlap"
            elif f == "gate_local_max":
                assert 1 <= v <= 8
            elif f == "aux_cus":
                assert v % 32 == 0 and mode == "overlap"
        assert e["ms_per_layer"] <= e["default_ms_per_layer"]
