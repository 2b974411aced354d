"""Host logic of the autotuner's table: class selection and the committed table's
shape (CPU only; the timing itself runs on the GPU)."""
import json
import os

from paper_2603_00035_amd import autotune as A


def _table(tmp_path, entries):
    p = str(tmp_path / "t.json")
    with open(p, "w") as f:
        json.dump({"entries": entries}, f)
    return p


def _entry(dt, max_nodes, th, kind="single"):
    return {"kind": kind, "dtype": dt, "max_nodes": max_nodes, "tuning": dict(A.DEFAULTS, tile_height=th)}


def test_lookup_picks_the_smallest_class_that_holds_the_grid(tmp_path):
    p = _table(tmp_path, [_entry("f32", 1 << 40, 64), _entry("f32", 1000, 32), _entry("f64", 5000, 32)])
    assert A.lookup(999, "f32", path=p).tile_height == 32
    assert A.lookup(1000, "f32", path=p).tile_height == 32
    assert A.lookup(1001, "f32", path=p).tile_height == 64
    assert A.lookup(4000, "f64", path=p).tile_height == 32
    assert A.lookup(6000, "f64", path=p) is None


def test_batch_entries_are_separate(tmp_path):
    p = _table(tmp_path, [_entry("f32", 1 << 40, 64), _entry("f32", 1 << 40, 32, kind="batch")])
    assert A.lookup(100, "f32", kind="single", path=p).tile_height == 64
    assert A.lookup(100, "f32", kind="batch", path=p).tile_height == 32


def test_missing_table_means_library_defaults(tmp_path):
    assert A.lookup(100, "f32", path=str(tmp_path / "absent.json")) is None


def test_committed_table_is_well_formed():
    if not os.path.exists(A.TABLE):
        return
    with open(A.TABLE) as f:
        t = json.load(f)
    assert t["knobs"] == list(A.KNOBS)
    for e in t["entries"]:
        assert e["dtype"] in ("f32", "f64") and e["kind"] in ("single", "batch")
        for k in A.KNOBS:
            assert e["tuning"][k] in A.CANDIDATES[k] or e["tuning"][k] == A.DEFAULTS[k]
