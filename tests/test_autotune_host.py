"""Host logic of the autotuner (no GPU): workload classes and the shape cache."""
import json

from paper_1304_5966_amd import autotune, swmi


def test_workload_classes_follow_mean_cells_per_pair():
    assert autotune.workload_class(1e6, 1) == swmi.TUNE_PAIR_SMALL
    assert autotune.workload_class(1e10 - 1, 1) == swmi.TUNE_PAIR_SMALL
    assert autotune.workload_class(1e10, 1) == swmi.TUNE_PAIR_LARGE
    assert autotune.workload_class(1e12 - 1, 1) == swmi.TUNE_PAIR_LARGE
    assert autotune.workload_class(2e13, 1) == swmi.TUNE_PAIR_HUGE
    # many small pairs form a batch; many large ones keep the class of one of them
    assert autotune.workload_class(2.76e11, 20_000) == swmi.TUNE_BATCH
    assert autotune.workload_class(6 * 6e12, 6) == swmi.TUNE_PAIR_HUGE
    assert autotune.workload_class(0.0, 0) == swmi.TUNE_PAIR_SMALL


def test_candidates_are_shapes_the_library_accepts():
    for R, w in autotune.CANDIDATES:
        assert R in (4, 6, 8)
        assert 1 <= w <= 16


def test_cache_round_trip_and_corrupt_file(tmp_path, monkeypatch):
    path = tmp_path / "sub" / "autotune.json"
    monkeypatch.setattr(autotune, "CACHE", str(path))
    assert autotune._load() == {}
    autotune._store("gfx950:256:batch", {"rows_per_lane": 6, "waves_per_cu": 16})
    autotune._store("gfx950:256:pair-huge", {"rows_per_lane": 8, "waves_per_cu": 8})
    data = json.loads(path.read_text())
    assert data == {"gfx950:256:batch": {"rows_per_lane": 6, "waves_per_cu": 16},
                    "gfx950:256:pair-huge": {"rows_per_lane": 8, "waves_per_cu": 8}}
    path.write_text("{not json")
    assert autotune._load() == {}


def test_band_candidates():
    from paper_1304_5966_amd import autotune
    c = autotune.band_candidates(4_000_000, 2048)
    assert c[0] == 0 and all(w % 64 == 0 for w in c[1:])
    assert 4_000_000 <= c[1] < 4_000_064  # one band
    assert c[2] * 3 >= 4_000_000 and c[3] * 4 >= 4_000_000
    # widths whose slots would exceed the memory cap are left out
    assert autotune.band_candidates(28_000_000, 2048) == [0]  # 7 Mi columns x 2049 slots > 96 GiB
    assert autotune.band_candidates(28_000_000, 512) == [0, 9_333_376, 7_000_000]
    assert autotune.band_candidates(100, 2048) == [0, 128, 64]

