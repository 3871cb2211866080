"""CPU tests of the schedule autotuner's host logic (bucketing, choice, table format)."""

import json

import pytest

from paper_2406_03726_amd import autotune as at


def test_bucketing():
    assert at.bucket_of(1000, 100, 3, 8) == (10, 1, 0)       # 2000 entries, degree 20
    assert at.bucket_of(1000, 100, 3, 0) == (9, 1, 0)        # directed: 1000 entries, degree 10
    assert at.bucket_of(1000, 10, 3, 8) == (10, 3, 0)        # degree 200
    assert at.bucket_of(1000, 40, 3, 8) == (10, 2, 0)        # degree 50
    assert at.bucket_of(10_000_000, 600_000, 50, 15)[2] == 1
    assert at.bucket_of(5, 1_000_000, 128, 15) == (3, 0, 2)
    assert at.bucket_of(0, 0, 1, 15) == (0, 0, 0)            # empty graph still has a bucket


def test_tune_picks_fastest_and_is_deterministic():
    shapes = [(100_000, 2000, 3, 15), (110_000, 2200, 3, 15), (1_000_000, 20000, 100, 15)]

    def fake_time(shape, sched):
        # best at 4096-entry parts for the smaller shapes, 16384 for the large one, and
        # 32-row buckets for K > 64 only
        target = 4096 if shape[0] < 500_000 else 16384
        sbt = 5 if shape[2] > 64 else 6
        return abs(sched["wave_entries"] - target) + (0.5 if sched["bucket_rows_log2"] != sbt else 0.0) + 1.0

    t = at.tune(shapes, fake_time)
    assert t.lookup(100_000, 2000, 3, 15) == {"wave_entries": 4096, "bucket_rows_log2": 6}
    assert t.lookup(1_000_000, 20000, 100, 15) == {"wave_entries": 16384, "bucket_rows_log2": 5}
    # ties resolve to the smaller candidate in sorted order
    t2 = at.tune([(100_000, 2000, 3, 15)], lambda s, c: 1.0)
    assert t2.lookup(100_000, 2000, 3, 15) == {"bucket_rows_log2": 5, "wave_entries": 2048}


def test_candidates_skip_equivalent_part_sizes():
    # 2000 entries: every part size holds the whole graph, so only the smallest is timed
    c = at.candidates("edge", 2000)
    assert {x["wave_entries"] for x in c} == {2048} and {x["bucket_rows_log2"] for x in c} == {5, 6}
    c = at.candidates("edge", 5000)
    assert {x["wave_entries"] for x in c} == {2048, 4096, 8192}
    assert len(at.candidates("edge")) == len(at.WAVE_ENTRIES) * len(at.BUCKET_SB)
    # resident CSR: the bucket kernels' candidates, then the CSR path's kernels'
    c = at.candidates("csr", 600)
    bk = [x for x in c if "bucket_rows_log2" in x]
    cp = [x for x in c if "waves_per_block" in x]
    assert len(bk) + len(cp) == len(c)
    assert bk == at.candidates("edge", 600)
    assert {x["wave_entries"] for x in cp} == {256, 512, 1024}
    assert {x["waves_per_block"] for x in cp} == set(at.CSR_WAVES_PER_BLOCK)


def test_csr_path_table_is_separate():
    shapes = [(200_000, 4000, 8, 7)]  # resident CSR: flags without symmetrization
    t = at.tune(shapes, lambda s, c: c["wave_entries"] / 1000 + c.get("waves_per_block", 10), path="csr")
    assert t.lookup(200_000, 4000, 8, 7, path="csr") == {"wave_entries": 256, "waves_per_block": 1}
    assert t.lookup(200_000, 4000, 8, 7) == {}  # nothing tuned for edge lists
    assert at.csr_shape((100_000, 4000, 8, 15)) == (200_000, 4000, 8, 7)
    with pytest.raises(ValueError):
        t.lookup(1, 1, 1, 0, path="nope")


def test_lookup_falls_back_to_nearest_and_default():
    t = at.ScheduleTable()
    t.entries[(10, 1, 0)] = {"wave_entries": 512}
    t.entries[(14, 1, 0)] = {"wave_entries": 2048}
    assert t.lookup(1000, 100, 3, 15) == {"wave_entries": 512}           # exact
    assert t.lookup(2 ** 11, 200, 3, 8) == {"wave_entries": 512}         # 2^12 entries: nearer 10
    assert t.lookup(2 ** 12 + 1, 400, 3, 8)["wave_entries"] in (512, 2048)
    assert t.lookup(2 ** 20, 100, 3, 8) == {}                            # other degree class
    assert t.lookup(1000, 100, 100, 15) == {}                            # other class-count class
    assert at.ScheduleTable().lookup(1, 1, 1, 0) == {}


def test_table_roundtrip_and_validation(tmp_path):
    t = at.ScheduleTable()
    t.entries[(12, 1, 1)] = {"wave_entries": 1024, "bucket_rows_log2": 6}
    t.csr_entries[(12, 1, 1)] = {"wave_entries": 512, "waves_per_block": 2}
    p = tmp_path / "t.json"
    t.save(str(p))
    t2 = at.ScheduleTable.load(str(p))
    assert t2.entries == t.entries and t2.csr_entries == t.csr_entries
    d = json.loads(p.read_text())
    d["entries"][0]["wave_entries"] = 300
    p.write_text(json.dumps(d))
    with pytest.raises(ValueError):
        at.ScheduleTable.load(str(p))
    d["version"] = 99
    p.write_text(json.dumps(d))
    with pytest.raises(ValueError):
        at.ScheduleTable.load(str(p))
    assert at.ScheduleTable.load(str(tmp_path / "missing.json")).entries == {}


def test_committed_table_is_valid():
    import os

    if os.path.exists(at.DEFAULT_TABLE):
        t = at.ScheduleTable.load(at.DEFAULT_TABLE)
        assert t.entries, "the committed table has no buckets"
