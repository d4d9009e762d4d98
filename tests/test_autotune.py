"""Host logic of the scan-tile autotuner (tests/test_gpu_autotune.py times it on the GPU):
size classes, the fastest candidate wins (ties to the taller band), one timing per class,
and the cache file round trip."""
import json

import paper_1705_03524_amd as swih
from paper_1705_03524_amd.autotune import Autotuner


def test_picks_fastest_and_caches(tmp_path):
    calls = []

    def timer(cfg, H, W):
        calls.append((cfg.band_rows, H, W))
        return {16: 3.0, 32: 1.0, 64: 2.0}[cfg.band_rows] * (H * W) / 1e5

    path = str(tmp_path / "tune.json")
    t = Autotuner(path, timer=timer)
    cfg = swih.Config(16, swih.MANHATTAN, [(31, 31)])
    assert t.best(cfg, 300, 200) == 32
    assert sorted(c[0] for c in calls) == [16, 32, 64]
    assert all((H, W) == (512, 256) for _, H, W in calls)   # timed at the size of the class
    assert t.best(cfg, 290, 250) == 32 and len(calls) == 3   # same class: no new timing
    t.best(cfg, 1000, 1000)
    assert len(calls) == 6
    saved = json.load(open(path))
    assert len(saved) == 2 and set(saved.values()) == {32}
    t2 = Autotuner(path, timer=lambda *a: 1 / 0)             # a fresh tuner reads the cache
    assert t2.best(cfg, 300, 200) == 32


def test_ties_prefer_taller_bands_and_sep_has_no_tiles(tmp_path):
    t = Autotuner(str(tmp_path / "t.json"), timer=lambda cfg, H, W: 1.0)
    assert t.best(swih.Config(8, swih.EUCLIDEAN, [(9, 9)]), 100, 100) == 64
    assert t.best(swih.Config(8, swih.GAUSSIAN_SEP, [(9, 9)]), 100, 100) == 0


def test_size_classes():
    assert Autotuner.size_class(100, 700) == (128, 1024)
    assert Autotuner.size_class(4000, 64) == (2048, 128)
