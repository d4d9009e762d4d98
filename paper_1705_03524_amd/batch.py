"""Batched SWIH: many frames (or crops), template queries and maps per launch.

Allocates the frames' workspaces from one device buffer, plans the batch with
the C ABI (host work), uploads the plan table, and launches the build, query
and map stages -- directly or as one captured HIP graph replayed per batch.
"""
from __future__ import annotations

import torch

from . import _swih as S

ALIGN = 256


class Batch:
    def __init__(self, cfg: S.Config, frames, queries=(), matches=(), device="cuda", ws=None):
        """frames: dicts with ``img`` (2-D uint8 device tensor or crop view) and
        optional ``scales`` and ``band_rows``; queries / matches as in
        ``_swih.batch_plan`` (their ``frame`` indexes ``frames``).  ``ws`` may
        supply the workspace buffer."""
        self.cfg = cfg
        offs, total = [], 0
        for f in frames:
            fc = S.Config(cfg.nbins, cfg.kernel, f.get("scales") or cfg.scales, cfg.gauss_terms,
                          band_rows=f.get("band_rows") or cfg.band_rows)
            nb = S.workspace_bytes(fc, f["img"].shape[0], f["img"].shape[1])
            offs.append((total, nb))
            total += (nb + ALIGN - 1) // ALIGN * ALIGN
        self.ws_bytes = total
        if ws is None:
            ws = torch.empty(max(total, ALIGN), dtype=torch.uint8, device=device)
        if ws.numel() < total or ws.data_ptr() % ALIGN:
            raise ValueError("workspace buffer too small or misaligned")
        self.ws = ws
        self.frames = [dict(f, ws=ws[o:o + nb]) for f, (o, nb) in zip(frames, offs)]
        self.queries = list(queries)
        self.matches = list(matches)
        self.h_table = S.batch_plan(cfg, self.frames, self.queries, self.matches)
        self.d_table = torch.from_numpy(self.h_table).to(device)
        if self.d_table.data_ptr() % ALIGN:
            raise RuntimeError("device table misaligned")
        self.graph = None
        self.status = None  # run_fused's status word

    def build(self, stream=None):
        S.batch_launch("build", self.h_table, self.d_table, stream)

    def query(self, stream=None):
        S.batch_launch("query", self.h_table, self.d_table, stream)

    def match(self, stream=None):
        S.batch_launch("match", self.h_table, self.d_table, stream)

    def run(self, stream=None):
        self.build(stream)
        self.query(stream)
        self.match(stream)

    def run_fused(self, stream=None, wait_ms: int = 0):
        """The whole batch in one persistent launch (swih_run_batch); the
        results equal ``run``'s bit for bit.  ``fused_status()`` tells whether
        every wait inside it was met."""
        if self.status is None:
            self.status = torch.zeros(1, dtype=torch.int32, device=self.d_table.device)
        S.batch_run(self.h_table, self.d_table, self.status, wait_ms, stream)

    def fused_status(self) -> int:
        """0 if every wait of the last run_fused was met (synchronises)."""
        return int(self.status.item()) if self.status is not None else 0

    def capture(self):
        """Capture build + query + match once in a HIP graph (torch.cuda.CUDAGraph)."""
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            self.run()  # warm-up outside capture
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.run()
        self.graph = g
        return g

    def replay(self):
        if self.graph is None:
            self.capture()
        self.graph.replay()
