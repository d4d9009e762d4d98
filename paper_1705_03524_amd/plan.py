"""Device-side plan: one workspace for an image size and configuration.

Thin convenience over the C ABI: it allocates the workspace with torch (the
library itself never allocates) and forwards every call to libswih.so.
"""
from __future__ import annotations

import torch

from . import _swih as S


class Plan:
    def __init__(self, cfg: S.Config, height: int, width: int, device="cuda", ws=None):
        self.cfg, self.H, self.W = cfg, int(height), int(width)
        self.nbytes = S.workspace_bytes(cfg, self.H, self.W)
        self.ws = ws if ws is not None else torch.empty(self.nbytes, dtype=torch.uint8, device=device)
        if self.ws.data_ptr() % 256:
            raise ValueError("workspace must be 256-byte aligned")
        if self.ws.numel() * self.ws.element_size() < self.nbytes:
            raise ValueError("workspace of %d bytes is smaller than the %d this plan needs"
                             % (self.ws.numel() * self.ws.element_size(), self.nbytes))
        self.device = self.ws.device

    @property
    def nplanes(self) -> int:
        """Stored planes per bin: 1 uniform, 3 Manhattan, 5 Euclidean, 5 for the Gaussian
        (its (2K+1)^2 weight terms contracted at the window corners, plus the count),
        2K+1 per axis for the separable Gaussian, 4 directions for the exponential."""
        if self.cfg.kernel == S.GAUSSIAN:
            return 5
        if self.cfg.kernel == S.GAUSSIAN_SEP:
            return 2 * self.cfg.K + 1
        return {S.UNIFORM: 1, S.MANHATTAN: 3, S.EUCLIDEAN: 5, S.EXPONENTIAL: 4}[self.cfg.kernel]

    @property
    def integer(self) -> bool:
        return self.cfg.kernel not in S.REAL_KINDS

    def valid_rect(self, scale_idx: int):
        w, h = self.cfg.scales[scale_idx]
        rx, ry = (w - 1) // 2, (h - 1) // 2
        return (rx, ry, self.W - 1 - rx, self.H - 1 - ry)

    def build(self, img, stream=None):
        S.build(self.cfg, img, self.ws, self.H, self.W, img.stride(0), stream)

    def query(self, scale_idx: int, centres, stream=None):
        """(normalised float [n, B], exact uint32 [n, B] or None) at int32 [n, 2] centres."""
        n = int(centres.shape[0])
        hist = torch.empty((n, self.cfg.nbins), dtype=torch.float32, device=self.device)
        raw = torch.empty((n, self.cfg.nbins), dtype=torch.uint32, device=self.device) if self.integer else None
        S.query(self.cfg, self.ws, self.H, self.W, scale_idx, centres, hist, raw, stream)
        return hist, raw

    def match(self, scale_idx: int, template=None, template_raw=None, rect=None, out=None, stream=None):
        r = rect if rect is not None else self.valid_rect(scale_idx)
        ny, nx = max(0, r[3] - r[1] + 1), max(0, r[2] - r[0] + 1)
        if out is None:
            out = torch.empty((ny, nx), dtype=torch.float32, device=self.device)
        S.match(self.cfg, self.ws, self.H, self.W, scale_idx, r, out, template, template_raw, stream)
        return out
