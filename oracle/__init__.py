"""CPU oracle for spatially weighted local histograms (SWIH).

TEST INFRASTRUCTURE ONLY -- only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no code
with the GPU path.

The brute-force part (``liboracle.so``, from ``swih_oracle.c``) evaluates every
window pixel by pixel: the convolution-style weighted histogram of Sec. 2 of the
paper, which the paper's SWIH method reproduces exactly (Sec. 3, Sec. 5).
``separable`` holds a second, independent route (per-bin separable
correlation) used only to cross-check the first.

Kernel kinds: 0 uniform, 1 Manhattan, 2 Euclidean (paraboloid), 3 Gaussian
(true Gaussian with sigma = window side / 4 unless given), 5 exponential
(exp(-|dx|/tx - |dy|/ty), tau = window side / 4 unless given).  See the C
file's header for the readings of the paper these fix.  For the two real-valued
kernels the ``sigma`` argument of every function is the pair of widths
(sigma or tau per axis).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

UNIFORM, MANHATTAN, EUCLIDEAN, GAUSSIAN, EXPONENTIAL = 0, 1, 2, 3, 5
KIND_NAMES = {UNIFORM: "uniform", MANHATTAN: "manhattan", EUCLIDEAN: "euclidean", GAUSSIAN: "gaussian",
              EXPONENTIAL: "exponential"}
REAL_KINDS = (GAUSSIAN, EXPONENTIAL)

_lib = None


def _load():
    global _lib
    if _lib is None:
        path = _build.build()
        lib = C.CDLL(path)
        i32, i64p, f64p, u8p, i32p = C.c_int, C.POINTER(C.c_int64), C.POINTER(C.c_double), \
            C.POINTER(C.c_uint8), C.POINTER(C.c_int32)
        lib.oracle_quantise.argtypes = [i32, i32]
        lib.oracle_set_threads.argtypes = [i32]
        lib.oracle_max_threads.restype = i32
        lib.oracle_kernel_table_int.argtypes = [i32, i32, i32, i64p]
        lib.oracle_kernel_table_gauss.argtypes = [i32, i32, C.c_double, C.c_double, f64p]
        lib.oracle_kernel_table_exp.argtypes = [i32, i32, C.c_double, C.c_double, f64p]
        lib.oracle_hist_i64.argtypes = [u8p, i32, i32, i32, i32, i64p, i32, i32, i32p, i32, i64p]
        lib.oracle_hist_f64.argtypes = [u8p, i32, i32, i32, i32, f64p, i32, i32, i32p, i32, f64p]
        lib.oracle_bc_i64.argtypes = [u8p, i32, i32, i32, i32, i64p, i32, i32, i64p, i32p, i32, f64p]
        lib.oracle_bc_f64.argtypes = [u8p, i32, i32, i32, i32, f64p, i32, i32, f64p, i32p, i32, f64p]
        lib.oracle_map_i64.argtypes = [u8p, i32, i32, i32, i32, i64p, i32, i32, i64p,
                                       i32, i32, i32, i32, f64p]
        lib.oracle_map_f64.argtypes = [u8p, i32, i32, i32, i32, f64p, i32, i32, f64p,
                                       i32, i32, i32, i32, f64p]
        _lib = lib
    return _lib


def _p(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


def set_threads(n: int):
    """Number of OpenMP threads the oracle's parallel loops use from now on."""
    _load().oracle_set_threads(int(n))


def threads() -> int:
    """Threads the oracle's next parallel loop will use."""
    return int(_load().oracle_max_threads())


def quantise(v, nbins: int):
    lib = _load()
    return lib.oracle_quantise(int(v), int(nbins))


def default_sigma(w: int, h: int):
    """Widths used throughout (Gaussian sigma, exponential tau): side / 4 per axis."""
    return w / 4.0, h / 4.0


def kernel_table(kind: int, w: int, h: int, sigma=None) -> np.ndarray:
    """Spatial kernel k[dy + ry, dx + rx] (int64, or float64 for the real-valued kernels)."""
    lib = _load()
    if kind in REAL_KINDS:
        sx, sy = sigma if sigma is not None else default_sigma(w, h)
        out = np.empty((h, w), np.float64)
        fn = lib.oracle_kernel_table_gauss if kind == GAUSSIAN else lib.oracle_kernel_table_exp
        if fn(w, h, float(sx), float(sy), _p(out, C.c_double)):
            raise ValueError("bad window %dx%d for kernel %d" % (w, h, kind))
        return out
    out = np.empty((h, w), np.int64)
    if lib.oracle_kernel_table_int(int(kind), w, h, _p(out, C.c_int64)):
        raise ValueError("bad kernel %r or window %dx%d" % (kind, w, h))
    return out


def mass(kind: int, w: int, h: int, sigma=None, table=None):
    """Kernel mass S = sum of the kernel table (int for integer kernels)."""
    t = table if table is not None else kernel_table(kind, w, h, sigma)
    return int(t.sum()) if t.dtype == np.int64 else float(t.sum())


# ---------------------------------------------------------------- wedding cake
# The discrete approximation of Sec. 2 (the wedding-cake approach, Fig. 4a): the
# window is cut into n nested windows R_0 (the whole window) > R_1 > ... >
# R_{n-1} around the centre; the rings R_i minus R_{i+1} get one weight each
# and the weighted ring histograms are summed.  Readings (the paper fixes
# neither): per axis the r + 1 distances 0..r from the centre are split into n
# equal runs, r_i = floor((r + 1)(n - i) / n) - 1 (so n = r + 1 gives one ring
# per distance; a negative half-size is an empty window), and each ring is
# weighted by the mean of the kernel over its own pixels, which keeps the
# total mass S.  The approximation is then a piecewise-constant kernel table,
# evaluated by the same brute force.

def cake_rings(w: int, h: int, n: int):
    """Half-sizes (rx_i, ry_i), i = 0..n-1, of the nested windows."""
    if n < 1:
        raise ValueError("ring count must be >= 1")
    rx, ry = (w - 1) // 2, (h - 1) // 2
    return [((rx + 1) * (n - i) // n - 1, (ry + 1) * (n - i) // n - 1) for i in range(n)]


def cake_ring_index(w: int, h: int, n: int) -> np.ndarray:
    """ring[dy + ry, dx + rx] = the largest i with |dx| <= rx_i and |dy| <= ry_i."""
    rx, ry = (w - 1) // 2, (h - 1) // 2
    ring = np.zeros((h, w), np.int64)
    for i, (ax, ay) in enumerate(cake_rings(w, h, n)):
        if ax < 0 or ay < 0:
            continue
        for dy in range(-ay, ay + 1):
            for dx in range(-ax, ax + 1):
                ring[dy + ry, dx + rx] = i
    return ring


def cake_table(kind: int, w: int, h: int, n: int, sigma=None) -> np.ndarray:
    """The wedding-cake kernel: every pixel of ring i weighted by the mean of the
    kernel over ring i (float64 [h, w])."""
    k = kernel_table(kind, w, h, sigma).astype(np.float64)
    ring = cake_ring_index(w, h, n)
    out = np.zeros((h, w), np.float64)
    for i in range(n):
        sel = ring == i
        if sel.any():
            out[sel] = k[sel].sum() / sel.sum()
    return out


def _img(img):
    a = np.ascontiguousarray(img, dtype=np.uint8)
    if a.ndim != 2:
        raise ValueError("image must be 2-D")
    return a


def hist(img, nbins: int, kind: int, w: int, h: int, centres, sigma=None, table=None) -> np.ndarray:
    """Raw weighted histograms H_b at the given centres ([n, 2] of (xc, yc)).

    int64 [n, nbins] for integer kernels, float64 for the real-valued ones.
    ``table`` overrides the kernel (any int64 or float64 h x w table).
    """
    lib = _load()
    a = _img(img)
    H, W = a.shape
    c = np.ascontiguousarray(np.asarray(centres, dtype=np.int32).reshape(-1, 2))
    tab = table if table is not None else kernel_table(kind, w, h, sigma)
    tab = np.ascontiguousarray(tab)
    n = c.shape[0]
    if tab.dtype == np.int64:
        out = np.empty((n, nbins), np.int64)
        rc = lib.oracle_hist_i64(_p(a, C.c_uint8), H, W, W, nbins, _p(tab, C.c_int64), w, h,
                                 _p(c, C.c_int32), n, _p(out, C.c_int64))
    else:
        tab = tab.astype(np.float64)
        out = np.empty((n, nbins), np.float64)
        rc = lib.oracle_hist_f64(_p(a, C.c_uint8), H, W, W, nbins, _p(tab, C.c_double), w, h,
                                 _p(c, C.c_int32), n, _p(out, C.c_double))
    if rc:
        raise ValueError("a centre puts the window outside the image")
    return out


def normalised(raw, kind: int, w: int, h: int, sigma=None, table=None) -> np.ndarray:
    """p_b = H_b / S (float64)."""
    return np.asarray(raw, np.float64) / float(mass(kind, w, h, sigma, table))


def template(img, nbins: int, kind: int, w: int, h: int, centre, sigma=None, table=None):
    """Template histogram at ``centre``: (raw, normalised)."""
    raw = hist(img, nbins, kind, w, h, [centre], sigma, table)[0]
    return raw, normalised(raw, kind, w, h, sigma, table)


def bc_at(img, nbins: int, kind: int, w: int, h: int, centres, tmpl, sigma=None, table=None) -> np.ndarray:
    """Bhattacharyya coefficient at listed centres against template ``tmpl``.

    Integer kernels take the raw integer template; the real-valued kernels take
    the normalised one.
    """
    lib = _load()
    a = _img(img)
    H, W = a.shape
    c = np.ascontiguousarray(np.asarray(centres, dtype=np.int32).reshape(-1, 2))
    n = c.shape[0]
    out = np.empty(n, np.float64)
    tab = np.ascontiguousarray(table if table is not None else kernel_table(kind, w, h, sigma))
    if tab.dtype == np.int64:
        t = np.ascontiguousarray(np.asarray(tmpl, np.int64))
        rc = lib.oracle_bc_i64(_p(a, C.c_uint8), H, W, W, nbins, _p(tab, C.c_int64), w, h,
                               _p(t, C.c_int64), _p(c, C.c_int32), n, _p(out, C.c_double))
    else:
        t = np.ascontiguousarray(np.asarray(tmpl, np.float64))
        rc = lib.oracle_bc_f64(_p(a, C.c_uint8), H, W, W, nbins, _p(tab, C.c_double), w, h,
                               _p(t, C.c_double), _p(c, C.c_int32), n, _p(out, C.c_double))
    if rc:
        raise ValueError("a centre puts the window outside the image")
    return out


def bc_map(img, nbins: int, kind: int, w: int, h: int, tmpl, rect=None, sigma=None, table=None) -> np.ndarray:
    """Dense likelihood map over the inclusive centre rectangle (x0, y0, x1, y1).

    Defaults to every valid centre.  Returns float64 [y1 - y0 + 1, x1 - x0 + 1].
    ``table`` overrides the kernel (a float64 table takes the normalised template).
    """
    lib = _load()
    a = _img(img)
    H, W = a.shape
    rx, ry = (w - 1) // 2, (h - 1) // 2
    x0, y0, x1, y1 = rect if rect is not None else (rx, ry, W - 1 - rx, H - 1 - ry)
    out = np.empty((max(0, y1 - y0 + 1), max(0, x1 - x0 + 1)), np.float64)
    tab = np.ascontiguousarray(table if table is not None else kernel_table(kind, w, h, sigma))
    if tab.dtype == np.int64:
        t = np.ascontiguousarray(np.asarray(tmpl, np.int64))
        rc = lib.oracle_map_i64(_p(a, C.c_uint8), H, W, W, nbins, _p(tab, C.c_int64), w, h,
                                _p(t, C.c_int64), x0, y0, x1, y1, _p(out, C.c_double))
    else:
        t = np.ascontiguousarray(np.asarray(tmpl, np.float64))
        rc = lib.oracle_map_f64(_p(a, C.c_uint8), H, W, W, nbins, _p(tab, C.c_double), w, h,
                                _p(t, C.c_double), x0, y0, x1, y1, _p(out, C.c_double))
    if rc:
        raise ValueError("centre rectangle outside the valid region")
    return out
