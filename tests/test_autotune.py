"""Host logic of the launch-shape autotuner (no GPU): candidates, keys, selection, cache."""
import json

from paper_2411_19588_amd import autotune as A
from paper_2411_19588_amd.rasterizer import RasterConfig


def test_candidates_are_valid_shapes():
    c = A.candidates()
    assert len(c) == len({json.dumps(x, sort_keys=True) for x in c})
    for s in c:
        assert s["tile"] in (8, 16)
        if s["tile"] == 8:
            assert s["pixels_per_lane"] == 1 and s["lds_batch"] == 64
        else:
            assert s["pixels_per_lane"] in (1, 2, 4) and s["lds_batch"] in (64, 256)
        assert s["record_fetch"] in ("lds", "scalar")


def test_key_buckets_workloads():
    k1 = A.workload_key("gfx950", 1_000_000, 3, [(1920, 1080)])
    k2 = A.workload_key("gfx950", 900_000, 3, [(1920, 1080)])
    k3 = A.workload_key("gfx950", 1_000_000, 3, [(1920, 1080)] * 2)
    assert k1 == k2 and k1 != k3


def test_tune_picks_fastest_and_caches(tmp_path):
    shapes = [dict(tile=16, pixels_per_lane=p, record_fetch="lds", lds_batch=256, persistent=False) for p in (1, 2, 4)]
    cost = {1: 3.0, 2: 1.5, 4: 2.0}
    calls = []

    def measure(cfg: RasterConfig):
        calls.append(cfg.pixels_per_lane)
        return cost[cfg.pixels_per_lane]

    path = str(tmp_path / "tune.json")
    base = RasterConfig(phases=2)
    got = A.tune(measure, base, shapes, path, "k")
    assert got.pixels_per_lane == 2 and got.phases == 2
    assert calls == [1, 2, 4]
    calls.clear()
    again = A.tune(measure, base, shapes, path, "k")            # served from the cache
    assert again.pixels_per_lane == 2 and calls == []
    assert json.load(open(path))["k"]["shape"]["pixels_per_lane"] == 2


def test_tune_skips_failing_shapes():
    shapes = [dict(tile=16, pixels_per_lane=p, record_fetch="lds", lds_batch=256, persistent=False) for p in (1, 4)]

    def measure(cfg):
        if cfg.pixels_per_lane == 1:
            raise RuntimeError("rejected")
        return 1.0

    assert A.tune(measure, RasterConfig(), shapes).pixels_per_lane == 4
    assert A.pick({0: None, 1: float("nan"), 2: 5.0, 3: 4.0}) == 3


def test_tune_all_tunes_shape_then_schedule():
    seen = []

    def measure(cfg):
        seen.append((cfg.pixels_per_lane, cfg.phases, cfg.phase0_shift))
        return (cfg.pixels_per_lane != 2) + abs(cfg.phase0_shift - 6) + 0.1 * cfg.phases

    got = A.tune_all(measure, RasterConfig())
    assert (got.pixels_per_lane, got.phases, got.phase0_shift) == (2, 2, 6)
    assert len(seen) == len(A.candidates()) + len(A.schedules())
