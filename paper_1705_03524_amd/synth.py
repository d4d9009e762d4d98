"""Seeded synthetic inputs for the SWIH hot path.

This module only draws images, regions and request streams.  It contains none
of the method's arithmetic (no quantiser, no spatial kernel, no integral
histogram, no similarity), so the CPU oracle and the HIP path can both be fed
from it without sharing any computation.

Every generator takes an explicit seed and uses numpy's PCG64 generator.

Workload recipes (the paper's own images -- the VOT2016 frame of its Fig. 5 and
the aerial imagery of its Fig. 7 -- are not available; these stand in for them):

* ``uniform_noise``: i.i.d. uniform intensities 0..255 (the 64x64 check image).
* ``smooth_noise``: uniform noise, blurred by a separable Gaussian FIR
  (radius 4 sigma, mirrored border), then stretched min..max onto 0..255 and
  rounded.  Without the stretch the blurred values crowd into a narrow band and
  most histogram bins stay empty.
* ``rect_scene``: ``smooth_noise`` plus axis-aligned bright (235) or dark (20)
  rectangles with sides drawn from 20..60, the synthetic stand-in for the
  paper's cluttered tracking scenes (Sec. 2, Fig. 3; Sec. 3, Fig. 5).
* ``track_sequence``: a moving target over a static ``smooth_noise``
  background, with distractors that carry exactly the target's pixel values in
  a different spatial arrangement (the target's values sorted by distance from
  its centre, handed out in reverse), so a plain histogram cannot tell them
  apart; the stand-in for the tracking imagery of Sec. 4 (Fig. 7).
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "rng",
    "uniform_noise",
    "smooth_noise",
    "rect_scene",
    "sample_centres",
    "odd",
    "batch_frames",
    "serving_requests",
    "track_sequence",
]


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def uniform_noise(seed: int, height: int, width: int) -> np.ndarray:
    """i.i.d. uniform uint8 intensities in [0, 255], shape (height, width)."""
    return rng(seed).integers(0, 256, size=(height, width), dtype=np.uint8)


def _blur_axis(a: np.ndarray, taps: np.ndarray, axis: int) -> np.ndarray:
    r = (len(taps) - 1) // 2
    pad = [(0, 0), (0, 0)]
    pad[axis] = (r, r)
    p = np.pad(a, pad, mode="symmetric")
    out = np.zeros_like(a)
    n = a.shape[axis]
    for k, t in enumerate(taps):
        sl = [slice(None), slice(None)]
        sl[axis] = slice(k, k + n)
        out += t * p[tuple(sl)]
    return out


def smooth_noise(seed: int, height: int, width: int, sigma: float = 3.0) -> np.ndarray:
    """Blurred uniform noise stretched onto the full 0..255 range (uint8)."""
    g = rng(seed)
    a = g.uniform(0.0, 256.0, size=(height, width))
    r = int(np.ceil(4.0 * sigma))
    t = np.arange(-r, r + 1, dtype=np.float64)
    taps = np.exp(-0.5 * (t / sigma) ** 2)
    taps /= taps.sum()
    a = _blur_axis(a, taps, 1)
    a = _blur_axis(a, taps, 0)
    lo, hi = a.min(), a.max()
    a = (a - lo) * (255.0 / max(hi - lo, 1e-12))
    return np.clip(np.rint(a), 0, 255).astype(np.uint8)


def rect_scene(seed: int, height: int, width: int, nrect: int = 6,
               side_lo: int = 20, side_hi: int = 60, sigma: float = 3.0):
    """Smooth noise plus ``nrect`` bright/dark rectangles drawn in order.

    Returns ``(image, rects)`` with ``rects`` a list of ``(x0, y0, w, h, value)``.
    """
    img = smooth_noise(seed, height, width, sigma)
    g = rng(seed + 7919)
    rects = []
    for _ in range(nrect):
        rw = int(g.integers(side_lo, side_hi + 1))
        rh = int(g.integers(side_lo, side_hi + 1))
        x0 = int(g.integers(0, max(1, width - rw + 1)))
        y0 = int(g.integers(0, max(1, height - rh + 1)))
        val = 235 if g.random() < 0.5 else 20
        img[y0:y0 + rh, x0:x0 + rw] = val
        rects.append((x0, y0, rw, rh, val))
    return img, rects


def odd(n: int) -> int:
    """Map a side length to the odd window size used for it (n -> n + 1 if even)."""
    n = int(n)
    return n if n % 2 == 1 else n + 1


def sample_centres(seed: int, height: int, width: int, w: int, h: int, n: int) -> np.ndarray:
    """``n`` seeded valid window centres (int32 [n, 2] as (xc, yc)).

    The four corners of the valid region and points on its four edges are
    always included, the rest is uniform over the valid region.
    """
    rx, ry = (w - 1) // 2, (h - 1) // 2
    x_lo, x_hi, y_lo, y_hi = rx, width - 1 - rx, ry, height - 1 - ry
    if x_hi < x_lo or y_hi < y_lo:
        return np.zeros((0, 2), np.int32)
    g = rng(seed)
    fixed = [(x_lo, y_lo), (x_hi, y_lo), (x_lo, y_hi), (x_hi, y_hi)]
    for _ in range(4):
        fixed.append((x_lo, int(g.integers(y_lo, y_hi + 1))))
        fixed.append((x_hi, int(g.integers(y_lo, y_hi + 1))))
        fixed.append((int(g.integers(x_lo, x_hi + 1)), y_lo))
        fixed.append((int(g.integers(x_lo, x_hi + 1)), y_hi))
    rest = max(0, n - len(fixed))
    xs = g.integers(x_lo, x_hi + 1, size=rest)
    ys = g.integers(y_lo, y_hi + 1, size=rest)
    pts = np.array(fixed + list(zip(xs.tolist(), ys.tolist())), dtype=np.int32)
    return pts[:max(n, 0)] if n < len(fixed) else pts


def batch_frames(seed: int, nframes: int = 64, w_range=(256, 1920), h_range=(256, 1080),
                 roi_range=(1, 8), side_range=(16, 128), scale_factors=(0.8, 1.0, 1.25)):
    """Uneven frame batch: frames of independent uniform sizes with target ROIs.

    Each frame is ``smooth_noise`` content.  Each ROI is a square of side
    ``s`` (made odd), centred uniformly so the window fits; its scales are
    ``odd(round(s * f))`` for ``f`` in ``scale_factors`` (clipped to the frame),
    and its search region is the 3s x 3s square around it, clipped to the
    frame.  Returns a list of dicts with ``image`` and ``rois``; each ROI is a
    dict with ``centre`` (x, y), ``scales`` [(w, h)], and ``search`` (x0, y0, x1, y1)
    as an inclusive pixel rectangle.
    """
    g = rng(seed)
    frames = []
    for f in range(nframes):
        W = int(g.integers(w_range[0], w_range[1] + 1))
        H = int(g.integers(h_range[0], h_range[1] + 1))
        img = smooth_noise(seed * 1000 + f + 1, H, W)
        nroi = int(g.integers(roi_range[0], roi_range[1] + 1))
        rois = []
        for _ in range(nroi):
            s = odd(int(g.integers(side_range[0], side_range[1] + 1)))
            scales = []
            for fac in scale_factors:
                m = min(W, H)
                largest_odd = m if m % 2 == 1 else m - 1
                sw = min(odd(max(3, int(round(s * fac)))), largest_odd)
                scales.append((sw, sw))
            smax = max(sc[0] for sc in scales)
            r = (smax - 1) // 2
            cx = int(g.integers(r, W - r))
            cy = int(g.integers(r, H - r))
            half = (3 * s) // 2
            search = (max(0, cx - half), max(0, cy - half), min(W - 1, cx + half), min(H - 1, cy + half))
            rois.append({"centre": (cx, cy), "scales": scales, "search": search})
        frames.append({"image": img, "rois": rois})
    return frames


FRAME_SIZES = ((640, 480), (1280, 720), (1920, 1080), (2560, 1440), (3840, 2160), (4096, 2160))


def serving_requests(seed: int, rate: float, n: int, nstreams: int = 16,
                     roi_range=(24, 96), search_mult=(2.0, 4.0),
                     scale_factors=(0.8, 1.0, 1.25), sizes=FRAME_SIZES):
    """Poisson stream of tracking requests from ``nstreams`` tracking streams.

    Inter-arrival times are exponential with mean ``1/rate`` seconds and
    requests go to the streams round-robin.  Each stream is one camera and
    one target: its frame size is drawn uniformly from ``sizes`` and its
    target side (made odd) from ``roi_range`` once, so its three window
    scales ``odd(round(s * f))`` stay fixed.  Per request the target centre is
    drawn uniformly where the largest window fits, and the search region is
    the square of side ``s * U[search_mult]`` (odd, at least the largest
    window) around it, clipped to the valid centres.
    """
    g = rng(seed)
    streams = []
    for _ in range(nstreams):
        W, H = sizes[int(g.integers(0, len(sizes)))]
        s = odd(int(g.integers(roi_range[0], roi_range[1] + 1)))
        scales = [(odd(max(3, int(round(s * f)))),) * 2 for f in scale_factors]
        streams.append(((H, W), s, scales))
    t = 0.0
    reqs = []
    for k in range(n):
        t += float(g.exponential(1.0 / rate))
        st = k % nstreams
        (H, W), s, scales = streams[st]
        smax = max(sc[0] for sc in scales)
        mult = float(g.uniform(*search_mult))
        side = odd(max(smax, int(round(s * mult))))
        r = (smax - 1) // 2
        cx = int(g.integers(r, W - r))
        cy = int(g.integers(r, H - r))
        half = (side - 1) // 2
        search = (max(r, cx - half), max(r, cy - half), min(W - 1 - r, cx + half), min(H - 1 - r, cy + half))
        reqs.append({"id": k, "t_arrive": t, "stream": st, "frame_hw": (H, W),
                     "centre": (cx, cy), "scales": scales, "search": search})
    return reqs


def _patch_pair(g: np.random.Generator, side: int):
    """A side x side target whose values rise toward its centre, and a distractor
    holding the same values (the same multiset) in reverse distance order."""
    r = (side - 1) // 2
    yy, xx = np.mgrid[-r:r + 1, -r:r + 1]
    dist = np.maximum(np.abs(xx), np.abs(yy)) + 0.01 * (np.abs(xx) + np.abs(yy))
    order = np.argsort(dist.ravel(), kind="stable")            # centre first
    vals = np.sort(g.integers(20, 256, size=side * side))[::-1]  # brightest first
    target = np.empty(side * side, np.int64)
    target[order] = vals
    distract = np.empty(side * side, np.int64)
    distract[order] = vals[::-1]
    return target.reshape(side, side).astype(np.uint8), distract.reshape(side, side).astype(np.uint8)


def track_sequence(seed: int, nframes: int = 60, height: int = 480, width: int = 640, side: int = 31,
                   ndistract: int = 2, speed: float = 4.0):
    """A synthetic tracking sequence.

    Returns ``(frames, truth, side)``: ``frames`` a list of uint8 (height,
    width) arrays, ``truth`` an int array [nframes, 2] of the target centre
    (x, y) per frame.  The target moves along a smooth curve (constant velocity
    plus a slow sway); each distractor follows its own curve and is drawn
    under the target where they overlap.
    """
    g = rng(seed)
    bg = smooth_noise(seed + 1, height, width, sigma=4.0) // 2 + 40   # low-contrast clutter
    target, distract = _patch_pair(g, side)
    r = (side - 1) // 2
    margin = r + 2

    def path(start, vel, amp, period):
        t = np.arange(nframes, dtype=np.float64)
        p = start[None, :] + vel[None, :] * t[:, None] + amp[None, :] * np.sin(2 * np.pi * t / period)[:, None]
        lo = np.array([margin, margin])
        hi = np.array([width - 1 - margin, height - 1 - margin])
        # fold the curve back into the frame
        span = hi - lo
        q = np.mod(p - lo, 2 * span)
        q = np.where(q > span, 2 * span - q, q)
        return np.rint(q + lo).astype(np.int64)

    def draw_dir():
        a = g.uniform(0, 2 * np.pi)
        return np.array([np.cos(a), np.sin(a)]) * speed

    start = np.array([g.uniform(width * 0.3, width * 0.7), g.uniform(height * 0.3, height * 0.7)])
    truth = path(start, draw_dir(), g.uniform(5, 15, size=2), g.uniform(20, 40))
    others = []
    for _ in range(ndistract):
        # distractors start a few sides away and cross the target's neighbourhood
        off = g.uniform(2.5, 4.0) * side * np.array([np.cos(g.uniform(0, 2 * np.pi)),
                                                     np.sin(g.uniform(0, 2 * np.pi))])
        others.append(path(start + off, draw_dir() * 0.8, g.uniform(5, 15, size=2), g.uniform(20, 40)))
    frames = []
    for f in range(nframes):
        img = bg.copy()
        for o in others:
            x, y = o[f]
            img[y - r:y + r + 1, x - r:x + r + 1] = distract
        x, y = truth[f]
        img[y - r:y + r + 1, x - r:x + r + 1] = target
        frames.append(img)
    return frames, truth, side
