"""A tracking loop around the likelihood maps (Sec. 4, the SWIFT idea without
LoFT's other features): per frame, the search region around the last position
is built once, each scale's likelihood map is computed against that scale's
template, the best window over all scales is the new position and scale, and
the templates move toward the histograms found there.

Every histogram and map comes from the library (swih_build, swih_query,
swih_match, swih_argmax); the loop itself only decides where to look next.
The same loop with the plain histogram (SWIH_UNIFORM) is the baseline of Sec. 4
(Fig. 7a against Fig. 7b).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import torch

from . import _swih as S
from .plan import Plan
from .synth import odd


@dataclass
class TrackState:
    centre: tuple          # (x, y) in frame coordinates
    side: int              # window side at scale 1
    scale: float = 1.0
    score: float = 1.0
    history: list = field(default_factory=list)


class Tracker:
    """One target.  ``kernel`` is any kernel of the library; ``scales`` are the
    relative window sizes searched per frame; ``search`` the half-size of the
    search region in window sides; ``alpha`` the template update rate."""

    def __init__(self, kernel, nbins: int = 16, scales=(0.9, 1.0, 1.1), search: float = 1.5,
                 alpha: float = 0.05, device="cuda"):
        self.kernel = S.KERNELS[kernel] if isinstance(kernel, str) else int(kernel)
        self.nbins, self.rel, self.search, self.alpha = nbins, tuple(scales), search, alpha
        self.device = device
        self.key = torch.zeros(1, dtype=torch.int64, device=device)
        self.ws = None
        self.templates = None
        self.state = None

    def _sides(self, side):
        return [odd(max(3, int(round(side * s)))) for s in self.rel]

    def _plan(self, H, W, sides):
        cfg = S.Config(self.nbins, self.kernel, [(s, s) for s in sides])
        n = S.workspace_bytes(cfg, H, W)
        if self.ws is None or self.ws.numel() < n:
            self.ws = torch.empty(n + 255, dtype=torch.uint8, device=self.device)
        return Plan(cfg, H, W, ws=self.ws[:n])

    def _box(self, frame, centre, side):
        H, W = frame.shape
        half = int(round(self.search * side)) + (max(self._sides(side)) - 1) // 2
        x0, x1 = max(0, centre[0] - half), min(W - 1, centre[0] + half)
        y0, y1 = max(0, centre[1] - half), min(H - 1, centre[1] + half)
        return x0, y0, x1, y1

    def init(self, frame, centre, side):
        """Templates at every scale from the target window at ``centre``."""
        sides = self._sides(side)
        x0, y0, x1, y1 = self._box(frame, centre, side)
        crop = frame[y0:y1 + 1, x0:x1 + 1]
        plan = self._plan(crop.shape[0], crop.shape[1], sides)
        plan.build(crop)
        c = torch.tensor([[centre[0] - x0, centre[1] - y0]], dtype=torch.int32, device=self.device)
        self.templates = [plan.query(k, c)[0][0].clone() for k in range(len(sides))]
        self.state = TrackState(tuple(int(v) for v in centre), int(side))

    def step(self, frame):
        """Localise the target in ``frame`` (a uint8 device tensor); returns the new state."""
        st = self.state
        side = int(round(st.side * st.scale))
        x0, y0, x1, y1 = self._box(frame, st.centre, side)
        crop = frame[y0:y1 + 1, x0:x1 + 1]
        Hc, Wc = crop.shape
        # a window larger than the search region (a target at the frame's edge)
        # is searched at the largest odd size that fits
        fit = min(Hc, Wc) if min(Hc, Wc) % 2 else min(Hc, Wc) - 1
        sides = [min(s, fit) for s in self._sides(side)]
        plan = self._plan(Hc, Wc, sides)
        plan.build(crop)
        best = None
        for k, s in enumerate(sides):
            m = plan.match(k, template=self.templates[k])
            S.argmax(m, self.key)
            idx, val = S.argmax_decode(int(self.key.item()))
            r = (s - 1) // 2
            cx, cy = x0 + r + idx % m.shape[1], y0 + r + idx // m.shape[1]
            if best is None or val > best[0]:
                best = (val, k, (cx, cy))
        val, k, (cx, cy) = best
        # the templates move toward the histograms at the new position
        c = torch.tensor([[cx - x0, cy - y0]], dtype=torch.int32, device=self.device)
        for j in range(len(sides)):
            h = plan.query(j, c)[0][0]
            self.templates[j].mul_(1.0 - self.alpha).add_(h, alpha=self.alpha)
        # the window size follows the best scale, within half to twice the first size
        st.scale = min(2.0, max(0.5, st.scale * self.rel[k] / self.rel[len(self.rel) // 2]))
        st.centre, st.score = (int(cx), int(cy)), float(val)
        st.history.append((st.centre, st.scale, st.score))
        return st


def run_sequence(kernel, frames, truth, side, nbins=16, device="cuda", **kw):
    """Track a synthetic sequence from its first ground-truth position.

    Returns a dict of per-frame centre errors (pixels), their mean and median,
    the fraction of frames within a quarter side of the truth, and the centres.
    """
    tr = Tracker(kernel, nbins=nbins, device=device, **kw)
    d = [torch.from_numpy(np.ascontiguousarray(f)).to(device) for f in frames]
    tr.init(d[0], tuple(int(v) for v in truth[0]), side)
    centres = [tuple(int(v) for v in truth[0])]
    for f in d[1:]:
        centres.append(tr.step(f).centre)
    c = np.array(centres, np.float64)
    err = np.sqrt(((c - np.asarray(truth, np.float64)) ** 2).sum(1))
    return {"errors": err, "mean_error": float(err.mean()), "median_error": float(np.median(err)),
            "success": float((err <= side / 4.0).mean()), "centres": c}
