"""ctypes binding of libswih.so (argument marshalling only).

Every step of the hot path runs in the library's HIP kernels.  PyTorch is used
for device buffers (``tensor.data_ptr()``) and streams
(``torch.cuda.current_stream().cuda_stream``).  There is no fallback: if the
library is missing or the GPU is absent the calls raise.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field
from typing import Sequence

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libswih.so")

UNIFORM, MANHATTAN, EUCLIDEAN, GAUSSIAN, GAUSSIAN_SEP, EXPONENTIAL = 0, 1, 2, 3, 4, 5
KERNELS = {"uniform": UNIFORM, "manhattan": MANHATTAN, "euclidean": EUCLIDEAN, "gaussian": GAUSSIAN,
           "gaussian_sep": GAUSSIAN_SEP, "exponential": EXPONENTIAL}
SERIES_KINDS = (GAUSSIAN, GAUSSIAN_SEP)
# real-valued histograms (no exact integer outputs), one plane set per scale
REAL_KINDS = (GAUSSIAN, GAUSSIAN_SEP, EXPONENTIAL)

OK, ERR_INVALID, ERR_WORKSPACE, ERR_UNSUPPORTED, ERR_HIP, ERR_SCRATCH = 0, -1, -2, -3, -4, -5

EXPORTED = ("swih_workspace_bytes", "swih_build", "swih_build_carries", "swih_build_planes",
            "swih_query", "swih_match", "swih_batch_table_bytes", "swih_batch_plan",
            "swih_build_batch", "swih_query_batch", "swih_match_batch", "swih_gauss_terms",
            "swih_status_string", "swih_cake_query", "swih_cake_match", "swih_brute_match", "swih_argmax",
            "swih_match_noalloc", "swih_copy", "swih_run_batch")


class SwihError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__("%s failed: %s (%d)" % (what, status_string(status), status))
        self.status = status


class _Scale(C.Structure):
    _fields_ = [("w", C.c_int32), ("h", C.c_int32)]


class _Config(C.Structure):
    _fields_ = [("nbins", C.c_int32), ("kernel", C.c_int32), ("nscales", C.c_int32),
                ("scales", C.POINTER(_Scale)), ("gauss_terms", C.c_int32), ("flags", C.c_uint32),
                ("band_rows", C.c_int32)]


class _Rect(C.Structure):
    _fields_ = [("x0", C.c_int32), ("y0", C.c_int32), ("x1", C.c_int32), ("y1", C.c_int32)]


class _FrameDesc(C.Structure):
    _fields_ = [("d_img", C.c_void_p), ("height", C.c_int32), ("width", C.c_int32),
                ("pitch", C.c_int32), ("nscales", C.c_int32), ("scales", C.POINTER(_Scale)),
                ("d_ws", C.c_void_p), ("ws_bytes", C.c_size_t), ("band_rows", C.c_int32)]


class _QueryDesc(C.Structure):
    _fields_ = [("frame", C.c_int32), ("scale_idx", C.c_int32), ("d_centres", C.c_void_p),
                ("n", C.c_int32), ("d_hist", C.c_void_p), ("d_hist_raw", C.c_void_p)]


class _MatchDesc(C.Structure):
    _fields_ = [("frame", C.c_int32), ("scale_idx", C.c_int32), ("centres", _Rect),
                ("d_template", C.c_void_p), ("d_template_raw", C.c_void_p), ("d_map", C.c_void_p)]


_lib = None


def load():
    """Load libswih.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libswih.so not built: run `python -m paper_1705_03524_amd.build`")
    lib = C.CDLL(LIB_PATH)
    vp, i32, sz = C.c_void_p, C.c_int32, C.c_size_t
    cfgp = C.POINTER(_Config)
    lib.swih_workspace_bytes.argtypes = [cfgp, i32, i32]
    lib.swih_workspace_bytes.restype = C.c_int64
    lib.swih_build.argtypes = [cfgp, vp, i32, i32, i32, vp, sz, vp]
    lib.swih_build.restype = C.c_int
    for name in ("swih_build_carries", "swih_build_planes"):
        f = getattr(lib, name)
        f.argtypes = [cfgp, vp, i32, i32, i32, i32, vp, sz, vp]
        f.restype = C.c_int
    lib.swih_query.argtypes = [cfgp, vp, sz, i32, i32, i32, vp, i32, vp, vp, vp]
    lib.swih_query.restype = C.c_int
    for name in ("swih_match", "swih_match_noalloc"):
        f = getattr(lib, name)
        f.argtypes = [cfgp, vp, sz, i32, i32, i32, vp, vp, _Rect, vp, vp]
        f.restype = C.c_int
    lib.swih_batch_table_bytes.argtypes = [cfgp, C.POINTER(_FrameDesc), i32, i32, i32]
    lib.swih_batch_table_bytes.restype = C.c_int64
    lib.swih_batch_plan.argtypes = [cfgp, C.POINTER(_FrameDesc), i32, C.POINTER(_QueryDesc), i32,
                                    C.POINTER(_MatchDesc), i32, vp, sz]
    lib.swih_batch_plan.restype = C.c_int
    for name in ("swih_build_batch", "swih_query_batch", "swih_match_batch"):
        f = getattr(lib, name)
        f.argtypes = [vp, vp, vp]
        f.restype = C.c_int
    lib.swih_cake_query.argtypes = [cfgp, vp, sz, i32, i32, i32, i32, vp, i32, vp, vp]
    lib.swih_cake_query.restype = C.c_int
    lib.swih_cake_match.argtypes = [cfgp, vp, sz, i32, i32, i32, i32, vp, _Rect, vp, vp]
    lib.swih_cake_match.restype = C.c_int
    lib.swih_brute_match.argtypes = [cfgp, vp, i32, i32, i32, i32, vp, _Rect, vp, vp]
    lib.swih_brute_match.restype = C.c_int
    lib.swih_argmax.argtypes = [vp, C.c_int64, vp, vp]
    lib.swih_argmax.restype = C.c_int
    lib.swih_gauss_terms.argtypes = [i32, i32, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                     C.POINTER(C.c_double)]
    lib.swih_gauss_terms.restype = C.c_int
    lib.swih_run_batch.argtypes = [vp, vp, vp, C.c_int32, vp]
    lib.swih_run_batch.restype = C.c_int
    lib.swih_copy.argtypes = [vp, vp, sz, vp]
    lib.swih_copy.restype = C.c_int
    lib.swih_status_string.argtypes = [C.c_int]
    lib.swih_status_string.restype = C.c_char_p
    _lib = lib
    return lib


def status_string(status: int) -> str:
    return load().swih_status_string(int(status)).decode()


DEFAULT_GAUSS_TERMS = 3     # K used when a config's gauss_terms is 0


@dataclass
class Config:
    """Python mirror of ``swih_config``."""
    nbins: int
    kernel: int
    scales: Sequence[tuple] = ((15, 15),)
    gauss_terms: int = 0
    flags: int = 0
    band_rows: int = 0      # scan-tile rows: 0 = 64, else 16, 32 or 64 (see autotune)
    _c: _Config = field(default=None, init=False, repr=False)
    _arr: object = field(default=None, init=False, repr=False)

    def __post_init__(self):
        if isinstance(self.kernel, str):
            self.kernel = KERNELS[self.kernel]
        self.scales = tuple((int(w), int(h)) for w, h in self.scales)

    def c(self) -> _Config:
        arr = (_Scale * max(1, len(self.scales)))(*[_Scale(w, h) for w, h in self.scales])
        self._arr = arr
        self._c = _Config(int(self.nbins), int(self.kernel), len(self.scales),
                          C.cast(arr, C.POINTER(_Scale)), int(self.gauss_terms), int(self.flags),
                          int(self.band_rows))
        return self._c

    @property
    def K(self) -> int:
        """Terms of the Gaussian series per axis (the default when gauss_terms is 0)."""
        return int(self.gauss_terms) or DEFAULT_GAUSS_TERMS


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)


def workspace_bytes(cfg: Config, height: int, width: int) -> int:
    n = load().swih_workspace_bytes(C.byref(cfg.c()), int(height), int(width))
    if n < 0:
        raise SwihError(int(n), "swih_workspace_bytes")
    return int(n)


def build(cfg: Config, img, ws, height=None, width=None, pitch=None, stream=None):
    """swih_build on a uint8 device tensor ``img`` (rows x pitch) into ``ws`` (uint8)."""
    H = int(height if height is not None else img.shape[0])
    W = int(width if width is not None else img.shape[1])
    P = int(pitch if pitch is not None else img.stride(0))
    st = load().swih_build(C.byref(cfg.c()), _ptr(img), H, W, P, _ptr(ws), ws.numel() * ws.element_size(),
                           _stream(stream))
    if st != OK:
        raise SwihError(st, "swih_build")


def build_phase(cfg: Config, img, ws, phase: str, set_idx: int = 0, height=None, width=None,
                pitch=None, stream=None):
    """One build phase: ``phase`` = "carries" or "planes" (see swih_build_carries)."""
    H = int(height if height is not None else img.shape[0])
    W = int(width if width is not None else img.shape[1])
    P = int(pitch if pitch is not None else img.stride(0))
    fn = {"carries": load().swih_build_carries, "planes": load().swih_build_planes}[phase]
    st = fn(C.byref(cfg.c()), _ptr(img), H, W, P, int(set_idx), _ptr(ws),
            ws.numel() * ws.element_size(), _stream(stream))
    if st != OK:
        raise SwihError(st, "swih_build_" + phase)


def query(cfg: Config, ws, height: int, width: int, scale_idx: int, centres, hist=None,
          hist_raw=None, stream=None):
    """swih_query at int32 [n, 2] device ``centres``."""
    n = int(centres.shape[0]) if centres is not None else 0
    st = load().swih_query(C.byref(cfg.c()), _ptr(ws), ws.numel() * ws.element_size(), int(height),
                           int(width), int(scale_idx), _ptr(centres), n, _ptr(hist), _ptr(hist_raw),
                           _stream(stream))
    if st != OK:
        raise SwihError(st, "swih_query")


def match(cfg: Config, ws, height: int, width: int, scale_idx: int, rect, out, template=None,
          template_raw=None, stream=None):
    """swih_match over the inclusive centre rectangle ``rect`` = (x0, y0, x1, y1)."""
    r = _Rect(*[int(v) for v in rect])
    st = load().swih_match(C.byref(cfg.c()), _ptr(ws), ws.numel() * ws.element_size(), int(height),
                           int(width), int(scale_idx), _ptr(template), _ptr(template_raw), r,
                           _ptr(out), _stream(stream))
    if st != OK:
        raise SwihError(st, "swih_match")


def match_noalloc(cfg: Config, ws, height: int, width: int, scale_idx: int, rect, out, template=None,
                  template_raw=None, stream=None):
    """swih_match_noalloc: swih_match whose Gaussian accumulator is the
    library's static per-device scratch (nothing is allocated)."""
    r = _Rect(*[int(v) for v in rect])
    st = load().swih_match_noalloc(C.byref(cfg.c()), _ptr(ws), ws.numel() * ws.element_size(),
                                   int(height), int(width), int(scale_idx), _ptr(template),
                                   _ptr(template_raw), r, _ptr(out), _stream(stream))
    if st != OK:
        raise SwihError(st, "swih_match_noalloc")


def copy(dst, src, nbytes: int, stream=None):
    """swih_copy: ``nbytes`` bytes from tensor ``src`` to tensor ``dst`` (device
    or pinned host memory) with a kernel on ``stream``."""
    if nbytes > dst.numel() * dst.element_size() or nbytes > src.numel() * src.element_size():
        raise ValueError("copy of %d bytes exceeds a buffer" % nbytes)
    st = load().swih_copy(_ptr(dst), _ptr(src), int(nbytes), _stream(stream))
    if st != OK:
        raise SwihError(st, "swih_copy")


def cake_query(cfg: Config, ws, height: int, width: int, scale_idx: int, rings: int, centres, hist,
               stream=None):
    """swih_cake_query: wedding-cake histograms at int32 [n, 2] device ``centres``."""
    n = int(centres.shape[0])
    st = load().swih_cake_query(C.byref(cfg.c()), _ptr(ws), ws.numel() * ws.element_size(), int(height),
                                int(width), int(scale_idx), int(rings), _ptr(centres), n, _ptr(hist),
                                _stream(stream))
    if st != OK:
        raise SwihError(st, "swih_cake_query")


def cake_match(cfg: Config, ws, height: int, width: int, scale_idx: int, rings: int, rect, out, template,
               stream=None):
    """swih_cake_match over the inclusive centre rectangle ``rect``."""
    r = _Rect(*[int(v) for v in rect])
    st = load().swih_cake_match(C.byref(cfg.c()), _ptr(ws), ws.numel() * ws.element_size(), int(height),
                                int(width), int(scale_idx), int(rings), _ptr(template), r, _ptr(out),
                                _stream(stream))
    if st != OK:
        raise SwihError(st, "swih_cake_match")


def brute_match(cfg: Config, img, scale_idx: int, rect, out, template_raw, height=None, width=None,
                pitch=None, stream=None):
    """swih_brute_match: the brute-force map straight from the image."""
    H = int(height if height is not None else img.shape[0])
    W = int(width if width is not None else img.shape[1])
    P = int(pitch if pitch is not None else img.stride(0))
    r = _Rect(*[int(v) for v in rect])
    st = load().swih_brute_match(C.byref(cfg.c()), _ptr(img), H, W, P, int(scale_idx), _ptr(template_raw), r,
                                 _ptr(out), _stream(stream))
    if st != OK:
        raise SwihError(st, "swih_brute_match")


def argmax(values, key, stream=None):
    """swih_argmax of a float device tensor into ``key`` (a 1-element int64 device
    tensor read as uint64).  Decode with ``argmax_decode``."""
    st = load().swih_argmax(_ptr(values), int(values.numel()), _ptr(key), _stream(stream))
    if st != OK:
        raise SwihError(st, "swih_argmax")


def argmax_decode(key: int):
    """(index, value) from a swih_argmax key."""
    import struct
    k = int(key) & 0xFFFFFFFFFFFFFFFF
    value = struct.unpack("<f", struct.pack("<I", k >> 32))[0]
    return 0xFFFFFFFF - (k & 0xFFFFFFFF), value


def gauss_terms(n: int, K: int = 0):
    """(coefficients a_0..a_K, frequencies w_0..w_K in radians per pixel, worst
    normalised 2-D error) of the series g(t) = sum_k a_k cos(w_k t); K = 0 is
    the default."""
    K = int(K) or DEFAULT_GAUSS_TERMS
    a = (C.c_double * (K + 1))()
    om = (C.c_double * (K + 1))()
    e = C.c_double()
    st = load().swih_gauss_terms(int(n), K, a, om, C.byref(e))
    if st != OK:
        raise SwihError(st, "swih_gauss_terms")
    return list(a), list(om), float(e.value)


def batch_plan(cfg: Config, frames, queries, matches):
    """Plan a batch (host work only).

    frames: list of dicts with ``img`` (2-D uint8 device tensor, possibly a
    strided crop view), ``ws`` (uint8 device tensor), optional ``scales``.
    queries: dicts with ``frame``, ``scale_idx``, ``centres`` (int32 [n, 2]
    device), ``hist`` and/or ``hist_raw`` outputs.  matches: dicts with
    ``frame``, ``scale_idx``, ``rect``, ``template`` or ``template_raw``,
    ``out``.  Returns the host table as a numpy uint8 array.
    """
    import numpy as np
    lib = load()
    keep = []
    fd = (_FrameDesc * max(1, len(frames)))()
    for k, f in enumerate(frames):
        img = f["img"]
        sc = f.get("scales")
        arr = None
        if sc:
            arr = (_Scale * len(sc))(*[_Scale(int(w), int(h)) for w, h in sc])
            keep.append(arr)
        fd[k] = _FrameDesc(img.data_ptr(), int(img.shape[0]), int(img.shape[1]), int(img.stride(0)),
                           len(sc) if sc else 0, C.cast(arr, C.POINTER(_Scale)) if arr else None,
                           f["ws"].data_ptr(), f["ws"].numel(), int(f.get("band_rows", 0)))
    qd = (_QueryDesc * max(1, len(queries)))()
    for k, q in enumerate(queries):
        c = q["centres"]
        qd[k] = _QueryDesc(int(q["frame"]), int(q.get("scale_idx", 0)), c.data_ptr() if c.numel() else None,
                           int(c.shape[0]), q["hist"].data_ptr() if q.get("hist") is not None else None,
                           q["hist_raw"].data_ptr() if q.get("hist_raw") is not None else None)
    md = (_MatchDesc * max(1, len(matches)))()
    for k, m in enumerate(matches):
        md[k] = _MatchDesc(int(m["frame"]), int(m.get("scale_idx", 0)), _Rect(*[int(v) for v in m["rect"]]),
                           m["template"].data_ptr() if m.get("template") is not None else None,
                           m["template_raw"].data_ptr() if m.get("template_raw") is not None else None,
                           m["out"].data_ptr())
    c = cfg.c()
    n = lib.swih_batch_table_bytes(C.byref(c), fd, len(frames), len(queries), len(matches))
    if n < 0:
        raise SwihError(int(n), "swih_batch_table_bytes")
    table = np.zeros(int(n), np.uint8)
    st = lib.swih_batch_plan(C.byref(c), fd, len(frames), qd, len(queries), md, len(matches),
                             table.ctypes.data_as(C.c_void_p), table.nbytes)
    if st != OK:
        raise SwihError(st, "swih_batch_plan")
    return table


def batch_run(h_table, d_table, status=None, wait_ms: int = 0, stream=None):
    """swih_run_batch: the whole planned batch in one persistent launch;
    ``status`` (int32 device tensor or None) receives 0 if every wait was met."""
    st = load().swih_run_batch(h_table.ctypes.data_as(C.c_void_p), C.c_void_p(d_table.data_ptr()),
                               _ptr(status), int(wait_ms), _stream(stream))
    if st != OK:
        raise SwihError(st, "swih_run_batch")


def batch_launch(which: str, h_table, d_table, stream=None):
    """``which`` = "build", "query" or "match": launch that part of a planned batch."""
    fn = {"build": load().swih_build_batch, "query": load().swih_query_batch,
          "match": load().swih_match_batch}[which]
    st = fn(h_table.ctypes.data_as(C.c_void_p), C.c_void_p(d_table.data_ptr()), _stream(stream))
    if st != OK:
        raise SwihError(st, "swih_%s_batch" % which)
