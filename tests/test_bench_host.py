"""Host logic of the benchmark line: the algorithmic byte model of the sweep
kernel and the matching of committed counter summaries to the layout a run
uses (so that a line never carries traffic measured on another layout or on
other kernel sources)."""

import copy
import json
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_sweep_bytes_per_update():
    # read S_i and chi_i, write I_i (3 values) and a 16 + 4 fp byte record
    # shared by the wavelengths
    assert bench.sweep_bytes_per_update(64, 4) == pytest.approx(12.0 + 32.0 / 64)
    assert bench.sweep_bytes_per_update(101, 4) == pytest.approx(12.0 + 32.0 / 101)
    assert bench.sweep_bytes_per_update(1, 8) == pytest.approx(24.0 + 48.0)


def _current(rec, files):
    """Whether a committed counter summary was taken on the kernel sources in the tree."""
    import hashlib

    h = hashlib.sha256()
    for f in files:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()[:16] == rec["source_sha256_16"]


def test_persistent_counters_match_layout_and_sources():
    rec = json.load(open(os.path.join(ROOT, "profiles", "persistent_sweep_c1_counters.json")))
    if not _current(rec, rec["sources"]):
        pytest.skip("the counter summary predates the current kernel sources (bench.py reports traffic null)")
    for e in rec["entries"]:
        lay = dict(e["layout"])
        got = bench.counter_traffic(64, 262144, "persistent", lay)
        assert got == e["sweep_bytes_per_launch"]["total"]
        # the bytes are FETCH_SIZE and WRITE_SIZE scaled by the copy calibration
        raw = e["raw_kib_per_launch"]
        assert got == pytest.approx(1024 * (raw["fetch"] * rec["fetch_scale"] + raw["write"] * rec["write_scale"]),
                                    rel=1e-4)
    # another workload, layout, row layout or launch mode has no measured traffic
    lay = dict(rec["entries"][0]["layout"])
    assert bench.counter_traffic(64, 262144, "persistent", dict(lay, shared_levels=0)) is None
    assert bench.counter_traffic(64, 262144, "persistent", dict(lay, interleave=0)) is None
    other_rows = "separate" if lay.get("rows", "separate") == "paired" else "paired"
    assert bench.counter_traffic(64, 262144, "persistent", dict(lay, rows=other_rows)) is None
    assert bench.counter_traffic(32, 262144, "persistent", lay) is None
    assert bench.counter_traffic(64, 1048576, "persistent", lay) is None


def test_counters_are_dropped_when_the_sources_change(tmp_path, monkeypatch):
    # a copy of the tree whose kernel source differs by one byte
    root = tmp_path / "repo"
    (root / "profiles").mkdir(parents=True)
    (root / "paper_2306_01041_amd" / "csrc").mkdir(parents=True)
    rec = json.load(open(os.path.join(ROOT, "profiles", "persistent_sweep_c1_counters.json")))
    if not _current(rec, rec["sources"]):
        pytest.skip("the counter summary predates the current kernel sources")
    (root / "profiles" / "persistent_sweep_c1_counters.json").write_text(json.dumps(rec))
    for f in ("k_persist.hip", "persist.h", "segment.h"):
        src = open(os.path.join(ROOT, "paper_2306_01041_amd", "csrc", f), "rb").read()
        (root / "paper_2306_01041_amd" / "csrc" / f).write_bytes(src)
    monkeypatch.setattr(bench, "ROOT", str(root))
    lay = dict(rec["entries"][0]["layout"])
    assert bench.counter_traffic(64, 262144, "persistent", lay) is not None
    seg = root / "paper_2306_01041_amd" / "csrc" / "segment.h"
    seg.write_bytes(seg.read_bytes() + b"\n")
    assert bench.counter_traffic(64, 262144, "persistent", lay) is None


@pytest.mark.parametrize("workload", ["c2", "c3"])
def test_level_step_counters_match_the_whole_layout(workload):
    rec = json.load(open(os.path.join(ROOT, "profiles", f"sweep_{workload}_counters.json")))
    if not _current(rec, rec["sources"]):
        pytest.skip("the counter summary predates the current kernel sources (bench.py reports traffic null)")
    lay = copy.deepcopy(rec["layout"])
    got = bench.lambda_counter_traffic(workload, "graph", lay)
    assert got == rec["sweep_bytes_per_formal_solution"]["total"]
    # measured traffic is at least the algorithmic bytes of the sweep
    updates = {"c2": 1048576 * 24 * 101, "c3": None}[workload]
    if updates:
        alg = bench.sweep_bytes_per_update(101, 4) * 104 / 101 * updates
        assert got > alg
    for key, other in (("pipeline", 0), ("interleave", 1), ("shared_levels", 0), ("xcd_chunks", 0),
                       ("rows", "separate" if lay.get("rows") == "paired" else "paired")):
        changed = dict(lay, **{key: other})
        assert bench.lambda_counter_traffic(workload, "graph", changed) is None, key
    assert bench.lambda_counter_traffic(workload, "persistent", lay) is None
