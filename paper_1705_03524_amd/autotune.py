"""Autotuner of the build's scan tiles.

A scan tile is 64 columns (one wave64 lane per column) by ``band_rows`` rows;
the rows are the free parameter (16, 32 or 64).  Short bands give more waves,
which fills the GPU on small frames and crops; tall bands keep the carries
small, which wins on large frames.  The best choice depends on the kernel, the
bin count and the frame size, so it is measured: per (device, kernel, bins,
series terms, size class) every candidate builds a synthetic frame of the
class's size (and, for the 2-D Gaussian, computes one map, since its lookups
cross band boundaries), the fastest candidate wins, and the choice is cached in
a JSON file so each class is timed once per device.

Integer results never depend on the choice; the real-valued kernels' results
change by rounding only (the tile-local origins move; measured at most 1.8e-7
on maps, asserted within 1e-5 by tests/test_gpu_autotune.py).
"""
from __future__ import annotations

import json
import os

from . import _swih as S

CANDIDATES = (16, 32, 64)
SIZE_CLASSES = (128, 256, 512, 1024, 2048)   # a side falls in the first class at least as long


def default_cache_path() -> str:
    return os.environ.get("SWIH_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "swih_autotune.json"))


class Autotuner:
    """``best(cfg, H, W)`` -> scan-tile rows.  ``timer(cfg, H, W)`` -> milliseconds
    may replace the GPU timing (the host-side logic is tested that way)."""

    def __init__(self, path: str | None = None, candidates=CANDIDATES, reps: int = 3, timer=None,
                 device="cuda"):
        self.path = path if path is not None else default_cache_path()
        self.candidates = tuple(candidates)
        self.reps = reps
        self.device = device
        self.on_gpu = timer is None
        self.timer = timer if timer is not None else self._time_gpu
        self.table = {}
        self.timings = {}
        if self.path and os.path.exists(self.path):
            try:
                with open(self.path) as f:
                    self.table = json.load(f)
            except (OSError, ValueError):
                self.table = {}

    @staticmethod
    def size_class(H: int, W: int):
        def up(n):
            for c in SIZE_CLASSES:
                if n <= c:
                    return c
            return SIZE_CLASSES[-1]
        return (up(H), up(W))

    def _device_name(self) -> str:
        if not self.on_gpu:
            return "host-timer"
        import torch
        return torch.cuda.get_device_name(torch.device(self.device))

    def key(self, cfg: S.Config, H: int, W: int) -> str:
        ch, cw = self.size_class(H, W)
        w, h = cfg.scales[0]
        return "%s|k%d|b%d|K%d|%dx%d|w%dx%d" % (self._device_name(), cfg.kernel, cfg.nbins,
                                               cfg.K, cw, ch, w, h)

    def best(self, cfg: S.Config, H: int, W: int) -> int:
        if cfg.kernel == S.GAUSSIAN_SEP:
            return 0                      # no scan tiles
        k = self.key(cfg, H, W)
        if k not in self.table:
            ch, cw = self.size_class(H, W)    # the class is timed at its own size
            times = {}
            for rows in self.candidates:
                c = S.Config(cfg.nbins, cfg.kernel, [cfg.scales[0]], cfg.gauss_terms, band_rows=rows)
                times[rows] = float(self.timer(c, ch, cw))
            self.timings[k] = times
            self.table[k] = min(times, key=lambda r: (times[r], -r))   # ties: the taller band
            self._save()
        return int(self.table[k])

    def _save(self):
        if not self.path:
            return
        try:
            os.makedirs(os.path.dirname(self.path) or ".", exist_ok=True)
            tmp = self.path + ".tmp%d" % os.getpid()
            with open(tmp, "w") as f:
                json.dump(self.table, f, indent=1, sort_keys=True)
            os.replace(tmp, self.path)
        except OSError:
            pass                          # the choice still holds for this process

    def _time_gpu(self, cfg: S.Config, H: int, W: int) -> float:
        """Milliseconds per build (+ one map for the 2-D Gaussian) of a synthetic
        frame, median of ``reps`` timed repetitions after one warm-up."""
        import torch

        from . import synth
        from .plan import Plan
        w, h = cfg.scales[0]
        w, h = min(w, W if W % 2 else W - 1), min(h, H if H % 2 else H - 1)
        cfg = S.Config(cfg.nbins, cfg.kernel, [(w, h)], cfg.gauss_terms, band_rows=cfg.band_rows)
        img = torch.from_numpy(synth.smooth_noise(H * 7 + W, H, W)).to(self.device)
        plan = Plan(cfg, H, W, device=self.device)
        t = torch.zeros(cfg.nbins, dtype=torch.float32, device=self.device)
        t[0] = 1.0

        def once():
            plan.build(img)
            if cfg.kernel == S.GAUSSIAN:
                plan.match(0, template=t)

        once()
        torch.cuda.synchronize()
        ts = []
        for _ in range(self.reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            once()
            b.record()
            torch.cuda.synchronize()
            ts.append(a.elapsed_time(b))
        del plan, img
        torch.cuda.empty_cache()
        return sorted(ts)[len(ts) // 2]
