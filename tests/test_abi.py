"""The C ABI loads, exports every symbol include/swih.h declares, and its host-only
paths (sizes, argument checks, the Gaussian series) behave -- no GPU needed."""
import math
import os
import re

import numpy as np
import pytest

import paper_1705_03524_amd as swih
from paper_1705_03524_amd import _swih

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    txt = open(os.path.join(ROOT, "include", "swih.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(swih_[a-z_0-9]+)\s*\(", txt)))


def test_library_exports_declared_symbols():
    lib = swih.load()
    names = declared_functions()
    assert len(names) >= 6
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(_swih.EXPORTED)


def test_status_strings():
    assert swih.status_string(0) == "ok"
    for s in (-1, -2, -3, -4):
        assert swih.status_string(s) != "unknown status"


def test_workspace_bytes_and_validation():
    cfg = swih.Config(16, swih.MANHATTAN, [(31, 31)])
    n = swih.workspace_bytes(cfg, 512, 512)
    planes = 3 * 16 * 513 * 512 * 4   # tile-major: 8 tiles of 64 columns, rows 0..512
    assert planes <= n < planes * 1.1
    bad = [swih.Config(0, swih.MANHATTAN, [(3, 3)]), swih.Config(257, swih.MANHATTAN, [(3, 3)]),
           swih.Config(8, 9, [(3, 3)]), swih.Config(8, swih.MANHATTAN, [(4, 3)]),
           swih.Config(8, swih.MANHATTAN, [(3, 3)], flags=1),
           swih.Config(8, swih.GAUSSIAN, [(3, 3)], gauss_terms=9),
           swih.Config(8, swih.MANHATTAN, [(601, 3)])]
    for c in bad:
        with pytest.raises(swih.SwihError) as e:
            swih.workspace_bytes(c, 512, 512)
        assert e.value.status == _swih.ERR_INVALID
    with pytest.raises(swih.SwihError):
        swih.workspace_bytes(cfg, 0, 10)
    # Gaussian keeps one plane set per scale
    g1 = swih.workspace_bytes(swih.Config(16, swih.GAUSSIAN, [(31, 31)]), 256, 256)
    g2 = swih.workspace_bytes(swih.Config(16, swih.GAUSSIAN, [(31, 31), (21, 21)]), 256, 256)
    assert g2 > 1.9 * g1 - 2e6


def test_plan_checks_a_given_workspace():
    torch = pytest.importorskip("torch")
    from paper_1705_03524_amd.plan import Plan
    cfg = swih.Config(8, swih.MANHATTAN, [(15, 15)])
    need = swih.workspace_bytes(cfg, 64, 64)
    buf = torch.empty(need + 512, dtype=torch.uint8)
    off = (-buf.data_ptr()) % 256
    with pytest.raises(ValueError, match="smaller"):
        Plan(cfg, 64, 64, ws=buf[off:off + need - 1])
    with pytest.raises(ValueError, match="aligned"):
        Plan(cfg, 64, 64, ws=buf[off + 1:off + 1 + need])
    assert Plan(cfg, 64, 64, ws=buf[off:off + need]).nbytes == need


def test_separable_workspace_and_validation():
    # one set per scale: H x W x B floats of row results (sized for any window)
    def a256(v):
        return (v + 255) // 256 * 256
    H, W, B = 480, 640, 16
    per_set = a256(H * W * B * 4)
    for scales in ([(31, 31)], [(31, 31), (9, 21), (101, 1)]):
        n = swih.workspace_bytes(swih.Config(B, swih.GAUSSIAN_SEP, scales), H, W)
        assert n == len(scales) * per_set
    two_d = swih.workspace_bytes(swih.Config(B, swih.GAUSSIAN, [(31, 31)]), H, W)
    # 5 corner-contracted planes + FP64 row carries + band-closing rows vs row results
    assert 5 * per_set < two_d < 8 * per_set
    for c in (swih.Config(8, swih.GAUSSIAN_SEP, [(3, 3)], gauss_terms=9),
              swih.Config(8, swih.GAUSSIAN_SEP, [(3, 3)], gauss_terms=-1),
              swih.Config(8, swih.GAUSSIAN_SEP, [(2, 3)]),
              swih.Config(8, 6, [(3, 3)])):
        with pytest.raises(swih.SwihError) as e:
            swih.workspace_bytes(c, 64, 64)
        assert e.value.status == _swih.ERR_INVALID


def test_exponential_workspace_and_host_checks():
    # per scale: 4 direction planes per bin (tile-major float) + double carries
    import ctypes as C

    def a256(v):
        return (v + 255) // 256 * 256
    H, W, B = 300, 200, 16
    NTX, NTY = (W + 63) // 64, (H + 63) // 64
    per_set = (a256(4 * B * NTX * (H + 1) * 64 * 4) + a256(4 * B * NTY * NTX * 64 * 8)
               + a256(4 * B * NTX * H * 8) + a256(4 * B * NTY * NTX * 8))
    for scales in ([(31, 31)], [(31, 31), (9, 21), (101, 1)]):
        assert swih.workspace_bytes(swih.Config(B, swih.EXPONENTIAL, scales), H, W) == len(scales) * per_set
    lib = swih.load()
    e = swih.Config(8, swih.EXPONENTIAL, [(5, 5)])
    st = lib.swih_query(C.byref(e.c()), C.c_void_p(256), 1 << 34, 64, 64, 0, C.c_void_p(256), 4,
                        None, C.c_void_p(256), None)
    assert st == _swih.ERR_UNSUPPORTED      # no exact raw histograms
    r = _swih._Rect(2, 2, 10, 10)
    st = lib.swih_match(C.byref(e.c()), C.c_void_p(256), 1 << 34, 64, 64, 0, None, C.c_void_p(256), r,
                        C.c_void_p(256), None)
    assert st == _swih.ERR_UNSUPPORTED      # raw template
    st = lib.swih_build_planes(C.byref(e.c()), C.c_void_p(256), 64, 64, 64, 1, C.c_void_p(256),
                               1 << 30, None)
    assert st == _swih.ERR_INVALID          # one set per scale: only set 0 exists
    st = lib.swih_build(C.byref(e.c()), C.c_void_p(256), 64, 64, 64, C.c_void_p(256), 16, None)
    assert st == _swih.ERR_WORKSPACE


def test_separable_host_checks():
    import ctypes as C
    lib = swih.load()
    g = swih.Config(8, swih.GAUSSIAN_SEP, [(5, 5)])
    st = lib.swih_query(C.byref(g.c()), C.c_void_p(256), 1 << 34, 64, 64, 0, C.c_void_p(256), 4,
                        None, C.c_void_p(256), None)
    assert st == _swih.ERR_UNSUPPORTED      # no exact raw histograms
    r = _swih._Rect(2, 2, 10, 10)
    st = lib.swih_match(C.byref(g.c()), C.c_void_p(256), 1 << 34, 64, 64, 0, None, C.c_void_p(256), r,
                        C.c_void_p(256), None)
    assert st == _swih.ERR_UNSUPPORTED      # raw template
    st = lib.swih_match(C.byref(g.c()), C.c_void_p(256), 16, 64, 64, 0, C.c_void_p(256), None, r,
                        C.c_void_p(256), None)
    assert st == _swih.ERR_WORKSPACE
    st = lib.swih_build_carries(C.byref(g.c()), C.c_void_p(256), 64, 64, 64, 1, C.c_void_p(256),
                                1 << 30, None)
    assert st == _swih.ERR_INVALID          # only set 0 exists


def test_host_checks_before_launch():
    # rejected on the host: nothing reaches the device, so no GPU is needed
    import ctypes as C
    lib = swih.load()
    cfg = swih.Config(8, swih.MANHATTAN, [(5, 5)])
    st = lib.swih_build(C.byref(cfg.c()), None, 64, 64, 64, None, 0, None)
    assert st == _swih.ERR_INVALID
    st = lib.swih_build(C.byref(cfg.c()), C.c_void_p(256), 64, 64, 32, C.c_void_p(256), 1 << 30, None)
    assert st == _swih.ERR_INVALID          # pitch < width
    st = lib.swih_build(C.byref(cfg.c()), C.c_void_p(256), 64, 64, 64, C.c_void_p(256), 16, None)
    assert st == _swih.ERR_WORKSPACE
    st = lib.swih_build(C.byref(cfg.c()), C.c_void_p(256), 64, 64, 64, C.c_void_p(300), 1 << 30, None)
    assert st == _swih.ERR_INVALID          # misaligned workspace
    r = _swih._Rect(1, 2, 10, 10)           # x0 < rx
    st = lib.swih_match(C.byref(cfg.c()), C.c_void_p(256), 1 << 30, 64, 64, 0, C.c_void_p(256), None, r,
                        C.c_void_p(256), None)
    assert st == _swih.ERR_INVALID
    r = _swih._Rect(2, 2, 10, 10)
    st = lib.swih_match(C.byref(cfg.c()), C.c_void_p(256), 1 << 30, 64, 64, 0, C.c_void_p(256),
                        C.c_void_p(256), r, C.c_void_p(256), None)
    assert st == _swih.ERR_INVALID          # both templates given
    g = swih.Config(8, swih.GAUSSIAN, [(5, 5)])
    st = lib.swih_query(C.byref(g.c()), C.c_void_p(256), 1 << 34, 64, 64, 0, C.c_void_p(256), 4,
                        None, C.c_void_p(256), None)
    assert st == _swih.ERR_UNSUPPORTED      # exact raw histograms are for integer kernels
    big = swih.Config(8, swih.EUCLIDEAN, [(2001, 2001)])
    st = lib.swih_build(C.byref(big.c()), C.c_void_p(256), 4000, 4000, 4000, C.c_void_p(256), 1 << 40, None)
    assert st == _swih.ERR_UNSUPPORTED      # kernel mass beyond 2^32
    st = lib.swih_query(C.byref(cfg.c()), C.c_void_p(256), 1 << 30, 64, 64, 0, None, 0, None, None, None)
    assert st == 0                          # n == 0 is a no-op


@pytest.mark.parametrize("n", [1, 3, 5, 7, 9, 15, 21, 31, 45, 63, 81, 121, 401])
def test_gauss_series_fidelity(n):
    # The series stands in for exp(-t^2 / (2 (n/4)^2)) on t in [-r, r]: check its
    # worst normalised 2-D histogram error from the coefficients and
    # frequencies alone, at the default K (3).
    a, om, err = swih.gauss_terms(n)
    assert len(a) == len(om) == 4
    r = (n - 1) // 2
    t = np.arange(-r, r + 1).astype(float)
    g = np.exp(-t ** 2 / (2 * (n / 4.0) ** 2))
    gt = sum(a[k] * np.cos(om[k] * t) for k in range(len(a)))
    k2 = np.outer(gt, gt) / gt.sum() ** 2 - np.outer(g, g) / g.sum() ** 2
    worst = max(k2[k2 > 0].sum(), -k2[k2 < 0].sum()) if n > 1 else 0.0
    assert worst == pytest.approx(err, rel=1e-6, abs=1e-15)
    assert err < 5e-8                       # 200x below the 1e-5 histogram bar
    assert om[0] == 0.0 and all(om[k] < om[k + 1] for k in range(len(om) - 1))
    assert sum(abs(v) for v in a) <= 2.0    # no cancelling coefficients


def test_gauss_series_orders():
    e = [swih.gauss_terms(31, K)[2] for K in (1, 2, 3, 4, 5)]
    assert all(e[i] > e[i + 1] for i in range(4)), e
    assert e[1] > 1e-5 > 1e-7 > e[2]        # K = 2 misses the bar, K = 3 meets it with margin


def test_gauss_series_fits_are_cached():
    # a fit runs once per (side, K) per process: later calls are lookups
    import time
    for n in (23, 57, 99):
        swih.gauss_terms(n)
    t = time.perf_counter()
    for _ in range(300):
        for n in (23, 57, 99):
            swih.gauss_terms(n)
    assert time.perf_counter() - t < 0.1       # ~5 us a lookup; a refit costs 0.2-1 ms


def test_gauss_series_beats_one_period():
    # free frequencies against harmonics of one integer period (the best
    # period's least-squares fit, by the same 2-D criterion): at least 100x
    # smaller worst error at K = 3
    n, K = 31, 3
    r = (n - 1) // 2
    t = np.arange(0, r + 1).astype(float)
    g = np.exp(-t ** 2 / (2 * (n / 4.0) ** 2))
    wt = np.where(t == 0, 1.0, math.sqrt(2.0))
    tt = np.arange(-r, r + 1).astype(float)
    gg = np.exp(-tt ** 2 / (2 * (n / 4.0) ** 2))
    best = np.inf
    for P in range(n, 6 * n + 1):
        om = 2 * math.pi * np.arange(K + 1) / P
        A = np.cos(np.outer(t, om))
        a = np.linalg.lstsq(A * wt[:, None], g * wt, rcond=None)[0]
        gt = np.cos(np.outer(np.abs(tt), om)) @ a
        k2 = np.outer(gt, gt) / gt.sum() ** 2 - np.outer(gg, gg) / gg.sum() ** 2
        best = min(best, max(k2[k2 > 0].sum(), -k2[k2 < 0].sum()))
    assert swih.gauss_terms(n, K)[2] * 100 < best


def test_baseline_host_checks():
    import ctypes as C
    lib = swih.load()
    r = _swih._Rect(2, 2, 10, 10)
    g = swih.Config(8, swih.GAUSSIAN, [(5, 5)])
    st = lib.swih_cake_query(C.byref(g.c()), C.c_void_p(256), 1 << 34, 64, 64, 0, 4, C.c_void_p(256), 4,
                             C.c_void_p(256), None)
    assert st == _swih.ERR_UNSUPPORTED      # the wedding cake needs an integer kernel's count plane
    m = swih.Config(8, swih.MANHATTAN, [(5, 5)])
    for rings in (0, 33):
        st = lib.swih_cake_match(C.byref(m.c()), C.c_void_p(256), 1 << 34, 64, 64, 0, rings, C.c_void_p(256),
                                 r, C.c_void_p(256), None)
        assert st == _swih.ERR_INVALID
    st = lib.swih_cake_match(C.byref(m.c()), C.c_void_p(256), 16, 64, 64, 0, 4, C.c_void_p(256), r,
                             C.c_void_p(256), None)
    assert st == _swih.ERR_WORKSPACE
    st = lib.swih_brute_match(C.byref(g.c()), C.c_void_p(256), 64, 64, 64, 0, C.c_void_p(256), r,
                              C.c_void_p(256), None)
    assert st == _swih.ERR_UNSUPPORTED      # exact integer kernels only
    bad = _swih._Rect(1, 2, 10, 10)         # x0 < rx
    st = lib.swih_brute_match(C.byref(m.c()), C.c_void_p(256), 64, 64, 64, 0, C.c_void_p(256), bad,
                              C.c_void_p(256), None)
    assert st == _swih.ERR_INVALID


def test_band_rows_validation_and_layout():
    base = swih.Config(16, swih.MANHATTAN, [(31, 31)])
    n64 = swih.workspace_bytes(base, 512, 512)
    for rows in (16, 32, 64):
        n = swih.workspace_bytes(swih.Config(16, swih.MANHATTAN, [(31, 31)], band_rows=rows), 512, 512)
        assert n >= n64 if rows < 64 else n == n64        # more bands, more carries; planes unchanged
    for rows in (8, 48, 128, -1):
        with pytest.raises(swih.SwihError):
            swih.workspace_bytes(swih.Config(16, swih.MANHATTAN, [(31, 31)], band_rows=rows), 512, 512)
