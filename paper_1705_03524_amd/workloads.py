"""Multi-frame tracking workloads: batched execution under an HBM budget.

A tracking step over many frames (Sec. 4: likelihood maps of several targets
per frame) becomes a list of *units*, each a frame or a search-region crop
with its window scales, plus per (target, scale) a template query at the
target centre and a likelihood map over the search region.

* Integer kernels: one unit per frame, holding every scale its targets use
  (one build serves all window sizes).
* Gaussian: one unit per (target, scale): the search-region crop plus the
  window margin, built with that scale's weight terms only.

``BatchedRunner`` packs units into sub-batches whose workspaces fit a byte
budget, plans each sub-batch once, and launches it with the batched C ABI
(directly or replayed from one captured HIP graph).  ``PerFrameRunner`` runs
the same units with the single-frame calls, one launch sequence per unit --
the plain per-frame GPU path.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import torch

from . import _swih as S
from . import synth
from .batch import ALIGN, Batch
from .plan import Plan


@dataclass
class Job:
    scale: tuple            # (w, h)
    centre: tuple           # template centre (unit coordinates)
    rect: tuple             # inclusive centre rectangle (unit coordinates)
    template: torch.Tensor = None
    template_raw: torch.Tensor = None
    out: torch.Tensor = None

    @property
    def windows(self) -> int:
        x0, y0, x1, y1 = self.rect
        return max(0, x1 - x0 + 1) * max(0, y1 - y0 + 1)


@dataclass
class Unit:
    img: torch.Tensor       # 2-D uint8 device view (frame or crop)
    scales: list
    jobs: list = field(default_factory=list)
    band_rows: int = 0      # scan-tile rows of this unit's build (0: the configuration's)


def _valid(rect, w, h, H, W):
    rx, ry = (w - 1) // 2, (h - 1) // 2
    x0, y0, x1, y1 = rect
    return (max(x0, rx), max(y0, ry), min(x1, W - 1 - rx), min(y1, H - 1 - ry))


def tracking_units(cfg: S.Config, frames, device="cuda"):
    """Units and jobs for ``synth.batch_frames``-style frames (dicts with
    ``image`` and ``rois`` of ``centre``, ``scales``, ``search``)."""
    units = []
    integer = cfg.kernel not in S.REAL_KINDS
    for fr in frames:
        img = torch.from_numpy(fr["image"]).to(device)
        H, W = fr["image"].shape
        if integer:
            scales = sorted({sc for r in fr["rois"] for sc in r["scales"]})
            u = Unit(img, scales)
            for r in fr["rois"]:
                for sc in r["scales"]:
                    rect = _valid(r["search"], sc[0], sc[1], H, W)
                    u.jobs.append(Job(sc, r["centre"], rect))
            units.append(u)
        else:
            for r in fr["rois"]:
                for sc in r["scales"]:
                    w, h = sc
                    rx, ry = (w - 1) // 2, (h - 1) // 2
                    x0, y0, x1, y1 = _valid(r["search"], w, h, H, W)
                    cx, cy = r["centre"]
                    # crop = search centres plus the window margin (and the template window)
                    ox0, oy0 = min(x0, cx) - rx, min(y0, cy) - ry
                    ox1, oy1 = max(x1, cx) + rx, max(y1, cy) + ry
                    crop = img[oy0:oy1 + 1, ox0:ox1 + 1]
                    u = Unit(crop, [sc])
                    u.jobs.append(Job(sc, (cx - ox0, cy - oy0), (x0 - ox0, y0 - oy0, x1 - ox0, y1 - oy0)))
                    units.append(u)
    for u in units:
        for j in u.jobs:
            x0, y0, x1, y1 = j.rect
            j.out = torch.empty((y1 - y0 + 1, x1 - x0 + 1), dtype=torch.float32, device=device)
            j.template = torch.empty(cfg.nbins, dtype=torch.float32, device=device)
            if integer:
                j.template_raw = torch.empty(cfg.nbins, dtype=torch.uint32, device=device)
    return units


def unit_config(cfg: S.Config, u: Unit) -> S.Config:
    return S.Config(cfg.nbins, cfg.kernel, u.scales, cfg.gauss_terms, band_rows=u.band_rows or cfg.band_rows)


def tune_units(cfg: S.Config, units, tuner) -> dict:
    """Set every unit's scan-tile rows from the autotuner; returns the choice per size class."""
    chosen = {}
    for u in units:
        H, W = u.img.shape
        u.band_rows = tuner.best(unit_config(cfg, u), H, W)
        chosen[tuner.size_class(H, W)] = u.band_rows
    return chosen


def unit_bytes(cfg: S.Config, u: Unit) -> int:
    nb = S.workspace_bytes(unit_config(cfg, u), u.img.shape[0], u.img.shape[1])
    return (nb + ALIGN - 1) // ALIGN * ALIGN


class BatchedRunner:
    """Units in sub-batches under ``budget`` workspace bytes; one shared buffer."""

    def __init__(self, cfg: S.Config, units, budget: int, device="cuda"):
        self.cfg, self.units = cfg, units
        groups, cur, cur_b = [], [], 0
        for u in units:
            nb = unit_bytes(cfg, u)
            if nb > budget:
                raise ValueError("a unit needs %d workspace bytes, above the budget %d" % (nb, budget))
            if cur and cur_b + nb > budget:
                groups.append(cur)
                cur, cur_b = [], 0
            cur.append(u)
            cur_b += nb
        if cur:
            groups.append(cur)
        self.ws = torch.empty(max(ALIGN, max(sum(unit_bytes(cfg, u) for u in g) for g in groups)),
                              dtype=torch.uint8, device=device)
        integer = cfg.kernel not in S.REAL_KINDS
        self.batches = []
        for g in groups:
            frames, queries, matches = [], [], []
            for fi, u in enumerate(g):
                frames.append({"img": u.img, "scales": u.scales, "band_rows": u.band_rows})
                for j in u.jobs:
                    si = u.scales.index(j.scale)
                    cen = torch.tensor([j.centre], dtype=torch.int32, device=device)
                    queries.append({"frame": fi, "scale_idx": si, "centres": cen,
                                    "hist": j.template.view(1, -1),
                                    "hist_raw": j.template_raw.view(1, -1) if integer else None})
                    m = {"frame": fi, "scale_idx": si, "rect": j.rect, "out": j.out}
                    if integer:
                        m["template_raw"] = j.template_raw
                    else:
                        m["template"] = j.template
                    matches.append(m)
            self.batches.append(Batch(cfg, frames, queries, matches, ws=self.ws))
        self.graph = None

    @property
    def nbatches(self):
        return len(self.batches)

    def run(self):
        for b in self.batches:
            b.run()

    def run_fused(self):
        """Each sub-batch in one persistent launch (swih_run_batch)."""
        for b in self.batches:
            b.run_fused()

    def fused_status(self) -> int:
        return max(b.fused_status() for b in self.batches)

    def capture(self):
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            self.run()
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self.run()

    def replay(self):
        if self.graph is None:
            self.capture()
        self.graph.replay()


class PerFrameRunner:
    """The same units with single-frame calls: build, then per job query + map."""

    def __init__(self, cfg: S.Config, units, budget: int, device="cuda"):
        self.cfg, self.units = cfg, units
        self.ws = torch.empty(max(ALIGN, max(unit_bytes(cfg, u) for u in units)), dtype=torch.uint8,
                              device=device)
        self.integer = cfg.kernel not in S.REAL_KINDS
        self.plans = []
        for u in units:
            uc = unit_config(cfg, u)
            nb = unit_bytes(cfg, u)
            self.plans.append(Plan(uc, u.img.shape[0], u.img.shape[1], ws=self.ws[:nb]))
        self.centres = [[torch.tensor([j.centre], dtype=torch.int32, device=device) for j in u.jobs]
                        for u in units]

    def run(self):
        for u, p, cens in zip(self.units, self.plans, self.centres):
            p.build(u.img)
            for j, c in zip(u.jobs, cens):
                si = u.scales.index(j.scale)
                S.query(p.cfg, p.ws, p.H, p.W, si, c, j.template.view(1, -1),
                        j.template_raw.view(1, -1) if self.integer else None)
                if self.integer:
                    S.match(p.cfg, p.ws, p.H, p.W, si, j.rect, j.out, template_raw=j.template_raw)
                else:
                    S.match(p.cfg, p.ws, p.H, p.W, si, j.rect, j.out, template=j.template)


def total_windows(units) -> int:
    return sum(j.windows for u in units for j in u.jobs)


def plane_bytes(cfg: S.Config, units) -> int:
    """Algorithmic bytes the builds write: 4 T B (H+1)(W+1) per plane set, or for
    the separable Gaussian 4 B H (W - w + 1) of row results per scale.  The
    Gaussian and the exponential keep one plane set per scale."""
    tot = 0
    for u in units:
        H, W = u.img.shape
        if cfg.kernel == S.GAUSSIAN_SEP:
            tot += sum(4 * cfg.nbins * H * (W - w + 1) for w, _ in u.scales)
            continue
        T = {S.UNIFORM: 1, S.MANHATTAN: 3, S.EUCLIDEAN: 5, S.EXPONENTIAL: 4, S.GAUSSIAN: 5}[cfg.kernel]
        nsets = len(u.scales) if cfg.kernel in (S.GAUSSIAN, S.EXPONENTIAL) else 1
        tot += nsets * 4 * T * cfg.nbins * (H + 1) * (W + 1)
    return tot


def batch_config_frames(seed: int, nframes: int = 64):
    """The uneven multi-frame batch: 64 frames of 256..1920 x 256..1080, 1..8
    targets of side 16..128 (odd), scales side * {0.8, 1, 1.25}, search 3s x 3s."""
    return synth.batch_frames(seed, nframes=nframes)
