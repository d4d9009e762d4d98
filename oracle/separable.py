"""Second CPU route to the same weighted histograms: per-bin separable correlation.

TEST INFRASTRUCTURE ONLY.  Used to cross-check the brute-force oracle, and
for full dense maps where brute force is slow.

Each kernel is written as a short sum of products of 1-D profiles,
k(dx, dy) = sum_r a_r(dx) * c_r(dy):

* uniform:   1 * 1
* Manhattan: (rx + ry + 1) * 1 * 1  -  |dx| * 1  -  1 * |dy|
* Euclidean: (rx^2 + ry^2 + 1) * 1 * 1  -  dx^2 * 1  -  1 * dy^2
* Gaussian:  exp(-dx^2 / 2 sx^2) * exp(-dy^2 / 2 sy^2)
* exponential: exp(-|dx| / tx) * exp(-|dy| / ty)

For every bin b the indicator image [Q(f) = b] is correlated along rows with
a_r and then along columns with c_r (numpy sliding windows and integer or
float matrix products), giving H_b at every valid centre in O(B H W (w + h)).
"""
from __future__ import annotations

import numpy as np
from numpy.lib.stride_tricks import sliding_window_view

UNIFORM, MANHATTAN, EUCLIDEAN, GAUSSIAN, EXPONENTIAL = 0, 1, 2, 3, 5


def profiles(kind: int, w: int, h: int, sigma=None):
    rx, ry = (w - 1) // 2, (h - 1) // 2
    dx = np.arange(-rx, rx + 1, dtype=np.int64)
    dy = np.arange(-ry, ry + 1, dtype=np.int64)
    one_x, one_y = np.ones_like(dx), np.ones_like(dy)
    if kind == UNIFORM:
        return [(one_x, one_y)]
    if kind == MANHATTAN:
        c = rx + ry + 1
        return [(c * one_x, one_y), (-np.abs(dx), one_y), (one_x, -np.abs(dy))]
    if kind == EUCLIDEAN:
        c = rx * rx + ry * ry + 1
        return [(c * one_x, one_y), (-dx * dx, one_y), (one_x, -dy * dy)]
    if kind == GAUSSIAN:
        sx, sy = sigma if sigma is not None else (w / 4.0, h / 4.0)
        gx = np.exp(-(dx.astype(np.float64) ** 2) / (2 * sx * sx))
        gy = np.exp(-(dy.astype(np.float64) ** 2) / (2 * sy * sy))
        return [(gx, gy)]
    if kind == EXPONENTIAL:
        tx, ty = sigma if sigma is not None else (w / 4.0, h / 4.0)
        return [(np.exp(-np.abs(dx) / tx), np.exp(-np.abs(dy) / ty))]
    raise ValueError(kind)


def hist_maps(img: np.ndarray, nbins: int, kind: int, w: int, h: int, sigma=None) -> np.ndarray:
    """H_b at every valid centre: array [nbins, H - h + 1, W - w + 1].

    int64 for integer kernels (exact), float64 for the real-valued ones.
    """
    img = np.asarray(img, np.uint8)
    H, W = img.shape
    q = (img.astype(np.int64) * nbins) // 256
    prof = profiles(kind, w, h, sigma)
    dt = np.float64 if kind in (GAUSSIAN, EXPONENTIAL) else np.int64
    out = np.zeros((nbins, H - h + 1, W - w + 1), dt)
    for b in range(nbins):
        m = (q == b).astype(dt)
        rows = sliding_window_view(m, w, axis=1)          # [H, W-w+1, w]
        for a, c in prof:
            t = rows @ a.astype(dt)                         # [H, W-w+1]
            cols = sliding_window_view(t, h, axis=0)        # [H-h+1, W-w+1, h]
            out[b] += cols @ c.astype(dt)
    return out
