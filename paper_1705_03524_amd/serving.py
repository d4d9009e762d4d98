"""Serving: continuous batching of tracking requests on one GPU.

A request names a tracking stream, a frame, a target centre, three window
scales and a search region (Sec. 4: likelihood maps of a target in the next
frame).  Per request and scale the server builds the Gaussian weighted
integral histograms of the search-region crop, takes the stream's template
histogram (computed on the stream's first request and kept resident on the
device), and computes the Bhattacharyya likelihood map of the search region;
the maps are copied to pinned host memory.  Latency runs from the request's
arrival to its maps being on the host.

``ContinuousServer``: requests that arrive while earlier ones are on the GPU
join the next micro-batch as soon as an in-flight slot and the HBM budget
allow; each micro-batch (crops uploaded, one batched build + query + map
launch sequence, maps downloaded) runs on its own stream, so micro-batches
overlap on the device.  ``SerialServer``: the plain path, one request at a
time with single-frame calls and a synchronisation per request.
"""
from __future__ import annotations

import gc
import time
from collections import deque
from contextlib import contextmanager

import numpy as np
import torch

from . import _swih as S
from .batch import ALIGN, Batch
from .plan import Plan


@contextmanager
def _no_gc_pauses():
    """Hold Python's cyclic collector off while requests are in flight (a
    collection of the many small objects a request loop makes can stall the
    loop for milliseconds); it runs once afterwards."""
    was = gc.isenabled()
    gc.disable()
    try:
        yield
    finally:
        if was:
            gc.enable()
        gc.collect()


class FramePool:
    """Host frames per frame size, shared by all requests of that size."""

    def __init__(self, sizes, make_image):
        self.frames = {}
        for (W, H) in sizes:
            self.frames[(H, W)] = np.ascontiguousarray(make_image(H, W))

    def get(self, hw) -> np.ndarray:
        return self.frames[tuple(hw)]


class Request:
    __slots__ = ("id", "t_arrive", "stream", "hw", "centre", "scales", "search", "crop_box",
                 "units", "maps", "host_maps", "t_done", "windows", "t_seen", "t_launch",
                 "t_launched", "slot", "batch_size", "marks")

    def __init__(self, r):
        self.id, self.t_arrive, self.stream = r["id"], r["t_arrive"], r["stream"]
        self.hw, self.centre, self.scales, self.search = r["frame_hw"], r["centre"], r["scales"], r["search"]
        self.t_done = None
        # host timestamps (seconds from the run's start): arrival noticed by the
        # loop, launch started, launch call returned; slot and micro-batch size
        self.t_seen = self.t_launch = self.t_launched = None
        self.slot = self.batch_size = None
        self.marks = None  # (label, host time) of each call inside a traced launch
        H, W = self.hw
        cx, cy = self.centre
        x0, y0, x1, y1 = self.search
        rmx = max((w - 1) // 2 for w, h in self.scales)
        rmy = max((h - 1) // 2 for w, h in self.scales)
        # the uploaded crop: search centres and the template centre plus the largest margin
        self.crop_box = (max(0, min(x0, cx) - rmx), max(0, min(y0, cy) - rmy),
                         min(W - 1, max(x1, cx) + rmx), min(H - 1, max(y1, cy) + rmy))
        ox, oy = self.crop_box[0], self.crop_box[1]
        self.units = []
        self.windows = 0
        for (w, h) in self.scales:
            rx, ry = (w - 1) // 2, (h - 1) // 2
            vx0, vy0 = max(x0, rx), max(y0, ry)
            vx1, vy1 = min(x1, W - 1 - rx), min(y1, H - 1 - ry)
            ux0, uy0 = min(vx0, cx) - rx - ox, min(vy0, cy) - ry - oy
            ux1, uy1 = max(vx1, cx) + rx - ox, max(vy1, cy) + ry - oy
            # (crop view box, template centre, map rectangle), all in the view's coordinates
            self.units.append(((ux0, uy0, ux1, uy1), (cx - ox - ux0, cy - oy - uy0),
                               (vx0 - ox - ux0, vy0 - oy - uy0, vx1 - ox - ux0, vy1 - oy - uy0)))
            self.windows += (vx1 - vx0 + 1) * (vy1 - vy0 + 1)


def unit_bytes(cfg, w, h, uh, uw):
    c = S.Config(cfg.nbins, cfg.kernel, [(w, h)], cfg.gauss_terms, band_rows=cfg.band_rows)
    nb = S.workspace_bytes(c, uh, uw)
    return (nb + ALIGN - 1) // ALIGN * ALIGN


def request_io(req: Request):
    """(crop bytes uploaded, map floats downloaded) of a request."""
    x0, y0, x1, y1 = req.crop_box
    return (x1 - x0 + 1) * (y1 - y0 + 1), req.windows


def request_bytes(cfg, req: Request) -> int:
    tot = 0
    for (w, h), (box, _, _) in zip(req.scales, req.units):
        tot += unit_bytes(cfg, w, h, box[3] - box[1] + 1, box[2] - box[0] + 1)
    return tot


def request_needs(cfg, req: Request):
    """What a request takes of a slot: (workspace bytes, crop bytes, map
    floats, staged centre ints)."""
    ib, of = request_io(req)
    return (request_bytes(cfg, req), ib, of, 2 * len(req.units))


def admit(needs, nfree, limits, max_batch, direct_single=True, busy=0, work_cap=None):
    """Admission of the waiting requests (``needs`` in arrival order, each a
    tuple of amounts, the first the workspace bytes) into ``nfree`` free slots
    whose capacities are ``limits`` (one per amount).  Returns the number of
    requests, taken in arrival order, that each successive free slot receives.

    * Light load (``direct_single`` and no more waiting requests than free
      slots): one request per slot.
    * Otherwise the waiting requests are spread over the free slots, an even
      share each (``ceil(waiting / free slots)``, at most ``max_batch``; every
      request to the first free slot when ``direct_single`` is off), a slot
      taking requests while they fit its capacities.
    * ``work_cap``: the workspace bytes of all micro-batches in flight
      (``busy`` of them already) stay within it, so large requests run one
      after another instead of sharing the memory bandwidth and all finishing
      late; a request still starts whenever nothing is in flight.
    A request that fits an empty slot is always admitted to one when nothing
    is in flight, so the loop makes progress; one that fits no slot is
    rejected before serving starts."""
    out = []
    k, n = 0, len(needs)
    cap = float("inf") if work_cap is None else work_cap

    def room(extra):
        return busy + extra <= cap or (busy == 0 and extra == needs[k][0])

    if direct_single and 0 < n <= nfree:
        while k < n and room(needs[k][0]):
            out.append(1)
            busy += needs[k][0]
            k += 1
        return out
    while k < n and len(out) < nfree:
        share = -(-(n - k) // (nfree - len(out))) if direct_single else max_batch
        used = [0] * len(limits)
        take = 0
        while k < n and take < min(share, max_batch):
            if any(u + a > c for u, a, c in zip(used, needs[k], limits)):
                break
            if not room(used[0] + needs[k][0]):
                break
            used = [u + a for u, a in zip(used, needs[k])]
            take += 1
            k += 1
        if take == 0:
            if busy > 0 or out:
                break  # the rest waits for work in flight to finish
            raise ValueError("request exceeds a slot's capacity")
        out.append(take)
        busy += used[0]
    return out


class _Templates:
    """Per tracking stream and scale: the template histogram, resident on the device,
    with the event of the launch that wrote it.  All templates live in one
    buffer allocated up front, so serving allocates no device memory (a new
    allocation on a slot's stream can stall the device for milliseconds)."""

    def __init__(self, nbins, device, capacity=4096):
        self.t = {}
        self.ready = {}
        self.nbins, self.device = nbins, device
        self.buf = torch.zeros((capacity, nbins), dtype=torch.float32, device=device)

    def get(self, stream, scale):
        key = (stream, scale)
        new = key not in self.t
        if new:
            k = len(self.t)
            if k >= self.buf.shape[0]:
                raise RuntimeError("more than %d (stream, scale) templates" % self.buf.shape[0])
            self.t[key] = self.buf[k:k + 1]
        return self.t[key], new

    def produced(self, stream, scale, event):
        self.ready[(stream, scale)] = event

    def event(self, stream, scale):
        return self.ready.get((stream, scale))


CENTRE_INTS = 4096  # template centres staged per slot (two ints per unit)


class _Slot:
    """One in-flight micro-batch's memory: workspace, pinned host staging for
    crops / template centres / maps and their device counterparts, a stream."""

    def __init__(self, budget, in_bytes, out_floats, device):
        self.ws = torch.empty(budget, dtype=torch.uint8, device=device)
        self.h_in = torch.empty(in_bytes, dtype=torch.uint8, pin_memory=True)
        self.d_in = torch.empty(in_bytes, dtype=torch.uint8, device=device)
        self.h_cen = torch.empty(CENTRE_INTS, dtype=torch.int32, pin_memory=True)
        self.d_cen = torch.empty(CENTRE_INTS, dtype=torch.int32, device=device)
        self.h_out = torch.empty(out_floats, dtype=torch.float32, pin_memory=True)
        self.d_out = torch.empty(out_floats, dtype=torch.float32, device=device)
        self.stream = torch.cuda.Stream()


class _MicroBatch:
    def __init__(self, reqs, stream, event):
        self.reqs, self.stream, self.event = reqs, stream, event
        self.work = 0  # workspace bytes of its requests


class ContinuousServer:
    def __init__(self, cfg: S.Config, pool: FramePool, budget: int, max_inflight: int = 3,
                 max_batch: int = 64, in_bytes: int = 64 << 20, out_floats: int = 32 << 20,
                 device="cuda", direct_single: bool = True, work_cap: int | None = None):
        """``direct_single``: while no more requests wait than there are free
        slots, each runs alone on its own slot with the single-unit calls (no
        batch table to plan and upload, the comb-form map); under heavier load
        the waiting requests are spread over the free slots as micro-batches
        (without it, they all go to one slot).  The maps are the same bit for
        bit either way.  ``work_cap``: optional bound on the workspace bytes in
        flight over all slots (see ``admit``); off by default, since at 2 GiB
        it left the server unable to keep up with 2000 requests/s."""
        self.cfg, self.pool, self.budget = cfg, pool, budget
        self.max_inflight, self.max_batch, self.device = max_inflight, max_batch, device
        self.direct_single = direct_single
        self.work_cap = work_cap
        self.in_bytes, self.out_floats = in_bytes, out_floats
        self.slots = [_Slot(budget, in_bytes, out_floats, device) for _ in range(max_inflight)]
        self.free = deque(range(max_inflight))
        self.templates = _Templates(cfg.nbins, device)
        self.trace = False  # record host timestamps of each call inside a launch (Request.marks)
        self._clock, self._t0 = time.perf_counter, 0.0

    def _launch(self, reqs, slot_id):
        cfg, dev = self.cfg, self.device
        sl = self.slots[slot_id]
        st = sl.stream
        frames, queries, matches = [], [], []
        produced, waits = [], []
        hin = sl.h_in.numpy()
        hcen = sl.h_cen.numpy()
        ioff, coff, ooff = 0, 0, 0
        crops, cens = [], []
        for r in reqs:  # stage crops and template centres in pinned memory
            x0, y0, x1, y1 = r.crop_box
            h, w = y1 - y0 + 1, x1 - x0 + 1
            np.copyto(hin[ioff:ioff + h * w].reshape(h, w), self.pool.get(r.hw)[y0:y1 + 1, x0:x1 + 1])
            crops.append((ioff, h, w))
            ioff += h * w
            cl = []
            for (_, tc, _) in r.units:
                hcen[coff:coff + 2] = tc
                cl.append(coff)
                coff += 2
            cens.append(cl)
        for r in reqs:
            self._mark(r, "staged")
        with torch.cuda.stream(st):
            S.copy(sl.d_in, sl.h_in, ioff, st)  # kernel copies: no copy-engine waits
            S.copy(sl.d_cen, sl.h_cen, 4 * coff, st)
            for r in reqs:
                self._mark(r, "upload")
            if len(reqs) == 1 and self.direct_single:
                return self._launch_direct(reqs[0], crops[0], cens[0], slot_id)
            for r, (io, h, w), cl in zip(reqs, crops, cens):
                crop = sl.d_in[io:io + h * w].view(h, w)
                r.maps = []
                for (sw, sh), (box, tc, rect), co in zip(r.scales, r.units, cl):
                    ux0, uy0, ux1, uy1 = box
                    fi = len(frames)
                    frames.append({"img": crop[uy0:uy1 + 1, ux0:ux1 + 1], "scales": [(sw, sh)]})
                    tmpl, new = self.templates.get(r.stream, (sw, sh))
                    if new:
                        queries.append({"frame": fi, "scale_idx": 0,
                                        "centres": sl.d_cen[co:co + 2].view(1, 2), "hist": tmpl})
                        produced.append((r.stream, (sw, sh)))
                    else:
                        ev = self.templates.event(r.stream, (sw, sh))
                        if ev is not None:
                            waits.append(ev)
                    rows, cols = rect[3] - rect[1] + 1, rect[2] - rect[0] + 1
                    m = sl.d_out[ooff:ooff + rows * cols].view(rows, cols)
                    r.maps.append((ooff, rows, cols))
                    ooff += rows * cols
                    matches.append({"frame": fi, "scale_idx": 0, "rect": rect, "template": tmpl[0],
                                    "out": m})
            b = Batch(cfg, frames, queries, matches, ws=sl.ws)
            for ev in waits:  # templates written by a batch on another stream
                st.wait_event(ev)
            b.build()
            b.query()
            if produced:
                tev = torch.cuda.Event()
                tev.record(st)
                for key in produced:
                    self.templates.produced(key[0], key[1], tev)
            b.match()
            S.copy(sl.h_out, sl.d_out, 4 * ooff, st)
            ev = torch.cuda.Event()
            ev.record(st)
        mb = _MicroBatch(reqs, slot_id, ev)
        mb.batch = b  # keep the plan table alive until done
        return mb

    def _mark(self, r, label):
        if self.trace:
            r.marks.append((label, self._clock() - self._t0))

    def _launch_direct(self, r, crop_io, cl, slot_id):
        """One request with single-unit calls on the slot's stream (the current
        stream here); its units run in stream order, so they share the slot's
        workspace."""
        cfg = self.cfg
        sl = self.slots[slot_id]
        st = sl.stream
        io, h, w = crop_io
        crop = sl.d_in[io:io + h * w].view(h, w)
        r.maps = []
        ooff = 0
        for (sw, sh), (box, tc, rect), co in zip(r.scales, r.units, cl):
            ux0, uy0, ux1, uy1 = box
            view = crop[uy0:uy1 + 1, ux0:ux1 + 1]
            uc = S.Config(cfg.nbins, cfg.kernel, [(sw, sh)], cfg.gauss_terms, band_rows=cfg.band_rows)
            nb = S.workspace_bytes(uc, view.shape[0], view.shape[1])
            p = Plan(uc, view.shape[0], view.shape[1], ws=sl.ws[:nb])
            self._mark(r, "plan")
            tmpl, new = self.templates.get(r.stream, (sw, sh))
            if not new:
                ev = self.templates.event(r.stream, (sw, sh))
                if ev is not None:  # written by a batch on another stream
                    st.wait_event(ev)
            p.build(view)
            self._mark(r, "build")
            if new:
                S.query(uc, p.ws, p.H, p.W, 0, sl.d_cen[co:co + 2].view(1, 2), tmpl)
                tev = torch.cuda.Event()
                tev.record(st)
                self.templates.produced(r.stream, (sw, sh), tev)
                self._mark(r, "query")
            rows, cols = rect[3] - rect[1] + 1, rect[2] - rect[0] + 1
            p.match(0, template=tmpl[0], rect=rect, out=sl.d_out[ooff:ooff + rows * cols].view(rows, cols))
            self._mark(r, "match")
            r.maps.append((ooff, rows, cols))
            ooff += rows * cols
        S.copy(sl.h_out, sl.d_out, 4 * ooff, st)
        self._mark(r, "download")
        ev = torch.cuda.Event()
        ev.record(st)
        self._mark(r, "event")
        mb = _MicroBatch([r], slot_id, ev)
        mb.batch = None
        return mb

    def _finish(self, mb):
        h_out = self.slots[mb.stream].h_out
        for r in mb.reqs:
            r.host_maps = [h_out[o:o + rows * cols].view(rows, cols).clone() for o, rows, cols in r.maps]

    def serve(self, requests, clock=time.perf_counter, keep_maps=False):
        """Run the arrival schedule in real time; returns the requests with t_done set."""
        with _no_gc_pauses():
            return self._serve(requests, clock, keep_maps)

    def _serve(self, requests, clock, keep_maps):
        reqs = [Request(r) for r in requests]
        # one small upload and download on every slot's stream before the
        # clock starts, so that first use of the copy kernel is not charged
        # to the first requests
        for sl in self.slots:
            S.copy(sl.d_in, sl.h_in, 256, sl.stream)
            S.copy(sl.h_out, sl.d_out, 256, sl.stream)
        torch.cuda.synchronize()
        limits = (self.budget, self.in_bytes, self.out_floats, CENTRE_INTS)
        for r in reqs:
            if any(a > c for a, c in zip(request_needs(self.cfg, r), limits)):
                raise ValueError("request %d exceeds a slot's capacity" % r.id)
        pending, inflight = deque(), deque()
        i, done, n = 0, 0, len(reqs)
        if self.trace:
            for r in reqs:
                r.marks = []
        t0 = clock()
        self._clock, self._t0 = clock, t0
        while done < n:
            now = clock() - t0
            while i < n and reqs[i].t_arrive <= now:
                reqs[i].t_seen = now
                pending.append(reqs[i])
                i += 1
            # every in-flight micro-batch is polled, not just the oldest: the
            # slots' streams finish out of order, and a small request must not
            # wait behind a large one launched before it
            running = deque()
            for mb in inflight:
                if not mb.event.query():
                    running.append(mb)
                    continue
                t = clock() - t0
                if keep_maps:
                    self._finish(mb)
                for r in mb.reqs:
                    r.t_done = t
                done += len(mb.reqs)
                self.free.append(mb.stream)
            inflight = running
            if pending and self.free:
                needs = [request_needs(self.cfg, r) for r in pending]
                limits = (self.budget, self.in_bytes, self.out_floats, CENTRE_INTS)
                busy = sum(mb.work for mb in inflight)
                k = 0
                for count in admit(needs, len(self.free), limits, self.max_batch, self.direct_single,
                                   busy, self.work_cap):
                    batch = [pending.popleft() for _ in range(count)]
                    slot = self.free.popleft()
                    t = clock() - t0
                    for r in batch:
                        r.t_launch, r.slot, r.batch_size = t, slot, count
                    mb = self._launch(batch, slot)
                    t = clock() - t0
                    for r in batch:
                        r.t_launched = t
                    mb.work = sum(nd[0] for nd in needs[k:k + count])
                    k += count
                    inflight.append(mb)
            elif not pending and i < n and not inflight:
                time.sleep(max(0.0, min(0.0005, reqs[i].t_arrive - (clock() - t0))))
        return reqs


class SerialServer:
    """One request at a time with the single-frame calls; synchronises per request."""

    def __init__(self, cfg: S.Config, pool: FramePool, budget: int, device="cuda"):
        self.cfg, self.pool, self.device = cfg, pool, device
        self.ws = torch.empty(budget, dtype=torch.uint8, device=device)
        self.templates = _Templates(cfg.nbins, device)

    def serve(self, requests, clock=time.perf_counter, keep_maps=False):
        with _no_gc_pauses():
            return self._serve(requests, clock, keep_maps)

    def _serve(self, requests, clock, keep_maps):
        reqs = [Request(r) for r in requests]
        cfg, dev = self.cfg, self.device
        t0 = clock()
        for r in reqs:
            wait = r.t_arrive - (clock() - t0)
            if wait > 0:
                time.sleep(wait)
            x0, y0, x1, y1 = r.crop_box
            crop = torch.from_numpy(np.ascontiguousarray(self.pool.get(r.hw)[y0:y1 + 1, x0:x1 + 1])).to(dev)
            maps = []
            for (w, h), (box, tc, rect) in zip(r.scales, r.units):
                ux0, uy0, ux1, uy1 = box
                view = crop[uy0:uy1 + 1, ux0:ux1 + 1]
                uc = S.Config(cfg.nbins, cfg.kernel, [(w, h)], cfg.gauss_terms, band_rows=cfg.band_rows)
                nb = S.workspace_bytes(uc, view.shape[0], view.shape[1])
                p = Plan(uc, view.shape[0], view.shape[1], ws=self.ws[:nb])
                p.build(view)
                tmpl, new = self.templates.get(r.stream, (w, h))
                if new:
                    S.query(uc, p.ws, p.H, p.W, 0, torch.tensor([tc], dtype=torch.int32, device=dev), tmpl)
                maps.append(p.match(0, template=tmpl[0], rect=rect))
            host = [m.cpu() for m in maps]  # synchronises
            if keep_maps:
                r.host_maps = host
            r.t_done = clock() - t0
        return reqs


def request_trace(reqs):
    """Per-request host timeline (ms from the run's start) of a served run."""
    ms = lambda v: None if v is None else round(v * 1e3, 4)
    return [{"id": r.id, "stream": r.stream, "arrive": ms(r.t_arrive), "seen": ms(r.t_seen),
             "launch": ms(r.t_launch), "launched": ms(r.t_launched), "done": ms(r.t_done),
             "slot": r.slot, "batch": r.batch_size, "windows": r.windows,
             "marks": [(k, ms(t)) for k, t in (r.marks or [])]} for r in reqs]


def latency_stats(reqs):
    lat = np.array([r.t_done - r.t_arrive for r in reqs]) * 1e3
    span = max(r.t_done for r in reqs) - min(r.t_arrive for r in reqs)
    wins = sum(r.windows for r in reqs)
    return {"p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "mean_ms": float(lat.mean()), "windows_per_s": wins / span, "requests": len(reqs),
            "achieved_req_per_s": len(reqs) / span}
