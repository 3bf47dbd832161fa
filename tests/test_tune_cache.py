"""The tuning cache (saved configurations, Section III): entries written by
rfim_tune_store are found by rfim_tune_lookup for exactly the same shapes and
steps, the file stays valid JSON, and malformed entries are rejected.  Host
code only (CPU)."""
from __future__ import annotations

import json

import pytest

import paper_2001_03389_amd as rf

STEPS = [("td", 3.25, "mean", 0), ("fd", 2.75, "mean", 32)]


def shapes_a():
    return [rf.shape_beam("u8", 1536, 12500), rf.shape_beam("f32", 4096, 8192)]


def test_missing_file_and_missing_key(tmp_path):
    p = str(tmp_path / "tune.json")
    assert rf.tune_lookup(p, shapes_a(), STEPS) is None
    rf.tune_store(p, shapes_a(), STEPS, (32, 81920, 64), 1.25)
    assert rf.tune_lookup(p, [rf.shape_beam("u8", 1536, 12500)], STEPS) is None


def test_round_trip_replace_and_json(tmp_path):
    p = str(tmp_path / "tune.json")
    rf.tune_store(p, shapes_a(), STEPS, (32, 81920, 64), 1.25)
    other = [rf.shape_beam("u8", 384, 25000, flags=True)]
    rf.tune_store(p, other, STEPS, (16, 40960, 8), 0.5)
    assert rf.tune_lookup(p, shapes_a(), STEPS) == (32, 81920, 64, 51200, 0, 4)
    assert rf.tune_lookup(p, other, STEPS) == (16, 40960, 8, 51200, 0, 4)
    rf.tune_store(p, shapes_a(), STEPS, (64, 163840, 8, 102400, 1, 8), 1.0)    # replaces
    assert rf.tune_lookup(p, shapes_a(), STEPS) == (64, 163840, 8, 102400, 1, 8)
    doc = json.load(open(p))
    assert len(doc) == 2
    assert all(set(v) >= {"u8_tile_cap", "f32_lds", "f32_tile_cap", "u8_lds", "u8_sched", "u8_td_rows", "ms"}
               for v in doc.values())


def test_entry_without_schedule_reads_as_default(tmp_path):
    """Cache entries written before the schedule and TD-rows parameters
    existed read as the two-pass schedule with four rows per work-group."""
    p = str(tmp_path / "tune.json")
    rf.tune_store(p, shapes_a(), STEPS, (32, 81920, 64, 51200, 1, 2), 1.0)
    txt = open(p).read().replace('"u8_sched": 1, ', "").replace('"u8_td_rows": 2, ', "")
    open(p, "w").write(txt)
    assert rf.tune_lookup(p, shapes_a(), STEPS) == (32, 81920, 64, 51200, 0, 4)


@pytest.mark.parametrize("variant", ["flags", "stride", "k-ulp", "replace", "bin", "order", "masked"])
def test_key_covers_shapes_and_steps(tmp_path, variant):
    p = str(tmp_path / "tune.json")
    rf.tune_store(p, shapes_a(), STEPS, (32, 81920, 64), 1.0)
    sh, st = shapes_a(), list(STEPS)
    if variant == "flags":
        sh[0] = rf.shape_beam("u8", 1536, 12500, flags=True)
    elif variant == "stride":
        sh[0] = rf.shape_beam("u8", 1536, 12500, row_stride=12512)
    elif variant == "k-ulp":
        st[0] = ("td", 3.2500000000000004, "mean", 0)
    elif variant == "replace":
        st[1] = ("fd", 2.75, "median", 32)
    elif variant == "bin":
        st[1] = ("fd", 2.75, "mean", 64)
    elif variant == "masked":
        st[0] = ("td_masked",) + tuple(st[0][1:])
    else:
        sh = sh[::-1]
    assert rf.tune_lookup(p, sh, st) is None


def test_malformed_entry_rejected(tmp_path):
    p = str(tmp_path / "tune.json")
    rf.tune_store(p, shapes_a(), STEPS, (32, 81920, 64), 1.0)
    txt = open(p).read().replace('"f32_lds": 81920', '"f32_lds": 12')
    open(p, "w").write(txt)
    with pytest.raises(rf.RfimError) as e:
        rf.tune_lookup(p, shapes_a(), STEPS)
    assert e.value.status == rf.RFIM_ERR_INVALID_ARG


def test_store_rejects_out_of_range(tmp_path):
    p = str(tmp_path / "tune.json")
    for bad in [(2, 81920, 64), (32, 10, 64), (32, 81920, 128), (32, 81920, 64, 100), (32, 81920, 64, 51200, 2),
                (32, 81920, 64, 51200, 0, 3)]:
        with pytest.raises(rf.RfimError):
            rf.tune_store(p, shapes_a(), STEPS, bad, 1.0)
