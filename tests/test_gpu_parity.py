"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Bar (stated per result):
* uniform / Manhattan / Euclidean raw histograms: bit-exact (integers);
* their likelihood maps from the exact integer template: (sum_b sqrt(H_b T_b)) / S
  in double, bins in order, rounded to float -- the same expression the oracle
  evaluates -- so equal bit for bit;
* Gaussian normalised histograms: within 1e-5 of the FP64 true-Gaussian oracle
  (error measured relative to the window mass, max over bins and windows);
* Gaussian maps: within 1e-5 of the oracle's map at every centre checked
  (tests/gpu_util.MAP_TOL), with the GPU's own template and with the oracle's.
"""
import numpy as np
import pytest

import oracle
from paper_1705_03524_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1705_03524_amd as swih  # noqa: E402
from paper_1705_03524_amd.plan import Plan  # noqa: E402

from gpu_util import GAUSS_TOL, MAP_TOL, all_centres, gauss_check, to_dev  # noqa: E402

INT_KINDS = (swih.UNIFORM, swih.MANHATTAN, swih.EUCLIDEAN)
GAUSS_KINDS = (swih.GAUSSIAN, swih.GAUSSIAN_SEP)


def run_int(img, nb, kind, w, h, tcentre, centres=None, rect=None):
    H, W = img.shape
    cfg = swih.Config(nb, kind, [(w, h)])
    plan = Plan(cfg, H, W)
    d_img = to_dev(img, torch)
    plan.build(d_img)
    c = centres if centres is not None else all_centres(H, W, w, h)
    hist, raw = plan.query(0, to_dev(c, torch))
    _, traw = plan.query(0, to_dev(np.array([tcentre], np.int32), torch))
    m = plan.match(0, template_raw=traw[0].contiguous(), rect=rect)
    torch.cuda.synchronize()
    return (raw.cpu().numpy().astype(np.int64), hist.cpu().numpy(), traw.cpu().numpy()[0].astype(np.int64),
            m.cpu().numpy())


# ---------------------------------------------------------------- 64 x 64 check image
def test_check_image_manhattan_15():
    print("case: 64x64 uniform noise, 8 bins, Manhattan 15x15, template (32, 32)", flush=True)
    img = synth.uniform_noise(0, 64, 64)
    raw, hist, traw, m = run_int(img, 8, swih.MANHATTAN, 15, 15, (32, 32))
    c = all_centres(64, 64, 15, 15)
    ref = oracle.hist(img, 8, oracle.MANHATTAN, 15, 15, c)
    assert np.array_equal(raw, ref)
    np.testing.assert_allclose(hist, ref / 1695.0, rtol=0, atol=6e-8)
    tref, _ = oracle.template(img, 8, oracle.MANHATTAN, 15, 15, (32, 32))
    assert np.array_equal(traw, tref)
    mref = oracle.bc_map(img, 8, oracle.MANHATTAN, 15, 15, tref)
    assert m.shape == (50, 50)
    assert np.array_equal(m, mref.astype(np.float32))
    assert m[25, 25] == 1.0


# ---------------------------------------------------------------- 512 x 512 scene
@pytest.fixture(scope="module")
def scene512():
    img, rects = synth.rect_scene(1, 512, 512)
    x0, y0, rw, rh, _ = rects[0]
    tc = (min(max(x0 + rw // 2, 15), 512 - 16), min(max(y0 + rh // 2, 15), 512 - 16))
    return img, tc


@pytest.mark.parametrize("kind", INT_KINDS)
def test_scene512_integer_kernels(scene512, kind):
    img, tc = scene512
    print("case: 512x512 scene, 16 bins, kind %d, 31x31, all windows" % kind, flush=True)
    raw, hist, traw, m = run_int(img, 16, kind, 31, 31, tc)
    c = all_centres(512, 512, 31, 31)
    ref = oracle.hist(img, 16, kind, 31, 31, c)
    assert np.array_equal(raw, ref)
    tref, _ = oracle.template(img, 16, kind, 31, 31, tc)
    mref = oracle.bc_map(img, 16, kind, 31, 31, tref)
    assert np.array_equal(m, mref.astype(np.float32))


# ---------------------------------------------------------------- ragged and degenerate
@pytest.mark.parametrize("kind", INT_KINDS)
@pytest.mark.parametrize("HW,nb,wh", [
    ((100, 77), 3, (5, 9)),
    ((65, 129), 16, (15, 15)),
    ((130, 64), 256, (3, 3)),
    ((70, 200), 1, (7, 61)),
    ((33, 33), 7, (33, 33)),      # one window covering the whole image
    ((20, 31), 5, (1, 1)),        # single-pixel window
    ((1, 90), 4, (9, 1)),         # one row
])
def test_ragged_integer(kind, HW, nb, wh):
    H, W = HW
    w, h = wh
    print("case: ragged %dx%d bins %d window %dx%d kind %d" % (H, W, nb, w, h, kind), flush=True)
    img = synth.uniform_noise(H * 1000 + W, H, W)
    c = all_centres(H, W, w, h)
    tc = tuple(c[len(c) // 2])
    raw, hist, traw, m = run_int(img, nb, kind, w, h, tc)
    ref = oracle.hist(img, nb, kind, w, h, c)
    assert np.array_equal(raw, ref)
    tref, _ = oracle.template(img, nb, kind, w, h, tc)
    mref = oracle.bc_map(img, nb, kind, w, h, tref)
    assert np.array_equal(m, mref.astype(np.float32))


# Both aggregate forms of the integer kernels: a plane set of at least 128
# (band, tile) blocks counts all bins at once in LDS histograms (up to 64 bins,
# 32 for the Euclidean's wider counters), smaller ones take a wave per bin.
# Ragged last bands and tiles; the last tile's 12 columns leave three of the
# four row-pass quarters empty.
@pytest.mark.parametrize("kind", INT_KINDS)
@pytest.mark.parametrize("HW,nb,band,wh", [
    ((300, 1100), 5, 16, (7, 9)),     # 342 blocks: histogram form
    ((300, 1100), 64, 16, (9, 5)),    # histogram form (Euclidean: per-bin, 64 bins)
    ((300, 1100), 32, 64, (15, 15)),  # 90 blocks: per-bin form
    ((517, 1100), 1, 32, (3, 17)),    # one bin, histogram form
    ((700, 1300), 16, 64, (31, 31)),  # 231 blocks of 64 rows, histogram form
])
def test_integer_aggregate_forms(kind, HW, nb, band, wh):
    H, W = HW
    w, h = wh
    print("case: aggregate forms %dx%d bins %d band %d window %dx%d kind %d" % (H, W, nb, band, w, h, kind),
          flush=True)
    img = synth.smooth_noise(H + W + nb, H, W) if nb >= 16 else synth.uniform_noise(H * 7 + W, H, W)
    plan = Plan(swih.Config(nb, kind, [(w, h)], band_rows=band), H, W)
    plan.build(to_dev(img, torch))
    c = all_centres(H, W, w, h)
    tc = tuple(int(v) for v in c[(len(c) * 3) // 7])
    _, raw = plan.query(0, to_dev(c, torch))
    _, traw = plan.query(0, to_dev(np.array([tc], np.int32), torch))
    m = plan.match(0, template_raw=traw[0].contiguous()).cpu().numpy()
    ref = oracle.hist(img, nb, kind, w, h, c)
    assert np.array_equal(raw.cpu().numpy().astype(np.int64), ref)
    tref, _ = oracle.template(img, nb, kind, w, h, tc)
    assert np.array_equal(m, oracle.bc_map(img, nb, kind, w, h, tref).astype(np.float32))


def test_sub_rectangle_and_pitch():
    # a crop inside a wider frame (row pitch > width) and a map over a sub-rectangle
    frame = synth.smooth_noise(4, 300, 400)
    crop = frame[37:237, 51:321]          # 200 x 270 view, pitch 400
    d_frame = to_dev(frame, torch)
    d_crop = d_frame[37:237, 51:321]
    cfg = swih.Config(16, swih.MANHATTAN, [(21, 15), (9, 9)])
    plan = Plan(cfg, 200, 270)
    plan.build(d_crop)
    rect = (30, 20, 140, 90)
    traw = plan.query(0, to_dev(np.array([[100, 60]], np.int32), torch))[1][0].contiguous()
    m = plan.match(0, template_raw=traw, rect=rect)
    m2 = plan.match(1, template_raw=plan.query(1, to_dev(np.array([[50, 50]], np.int32), torch))[1][0].contiguous())
    torch.cuda.synchronize()
    img = np.ascontiguousarray(crop)
    tref, _ = oracle.template(img, 16, oracle.MANHATTAN, 21, 15, (100, 60))
    assert np.array_equal(traw.cpu().numpy().astype(np.int64), tref)
    assert np.array_equal(m.cpu().numpy(), oracle.bc_map(img, 16, oracle.MANHATTAN, 21, 15, tref, rect=rect).astype(np.float32))
    tref2, _ = oracle.template(img, 16, oracle.MANHATTAN, 9, 9, (50, 50))
    assert np.array_equal(m2.cpu().numpy(), oracle.bc_map(img, 16, oracle.MANHATTAN, 9, 9, tref2).astype(np.float32))


def test_float_template_path_integer_kernel():
    img = synth.uniform_noise(9, 96, 80)
    cfg = swih.Config(8, swih.EUCLIDEAN, [(11, 13)])
    plan = Plan(cfg, 96, 80)
    plan.build(to_dev(img, torch))
    _, tp = oracle.template(img, 8, oracle.EUCLIDEAN, 11, 13, (40, 50))
    m = plan.match(0, template=to_dev(tp.astype(np.float32), torch))
    torch.cuda.synchronize()
    mref = oracle.bc_map(img, 8, oracle.EUCLIDEAN, 11, 13, oracle.template(img, 8, oracle.EUCLIDEAN, 11, 13, (40, 50))[0])
    # template rounded to float: error <= sum_b sqrt(p_b) |sqrt(t_b') - sqrt(t_b)|
    assert np.max(np.abs(m.cpu().numpy() - mref)) < 1e-6


def test_uint32_wrap_large_frame():
    # 4096 x 2160: sums of x (and x^2, y^2) per bin exceed 2^32 and wrap; the
    # window histograms must still be exact (arithmetic modulo 2^32).
    H, W = 2160, 4096
    img = synth.smooth_noise(21, H, W)
    print("case: 4096x2160 wrap, Manhattan + Euclidean 81x81, sampled", flush=True)
    c = synth.sample_centres(5, H, W, 81, 81, 2048)
    for kind in (swih.MANHATTAN, swih.EUCLIDEAN):
        cfg = swih.Config(16, kind, [(81, 81)])
        plan = Plan(cfg, H, W)
        plan.build(to_dev(img, torch))
        _, raw = plan.query(0, to_dev(c, torch))
        got = raw.cpu().numpy().astype(np.int64)
        ref = oracle.hist(img, 16, kind, 81, 81, c)
        assert np.array_equal(got, ref)
        del plan
        torch.cuda.empty_cache()


def test_max_side_uniform():
    H, W = 8192, 8192
    print("case: 8192x8192 uniform kernel 201x201, sampled", flush=True)
    img = synth.uniform_noise(3, H, W)
    c = synth.sample_centres(8, H, W, 201, 201, 512)
    cfg = swih.Config(4, swih.UNIFORM, [(201, 201)])
    plan = Plan(cfg, H, W)
    plan.build(to_dev(img, torch))
    _, raw = plan.query(0, to_dev(c, torch))
    ref = oracle.hist(img, 4, oracle.UNIFORM, 201, 201, c)
    assert np.array_equal(raw.cpu().numpy().astype(np.int64), ref)


def test_empty_inputs_are_noops():
    img = synth.uniform_noise(1, 40, 40)
    cfg = swih.Config(4, swih.MANHATTAN, [(5, 5)])
    plan = Plan(cfg, 40, 40)
    plan.build(to_dev(img, torch))
    h, r = plan.query(0, torch.empty((0, 2), dtype=torch.int32, device="cuda"))
    assert h.shape == (0, 4)
    out = torch.full((1,), 7.0, device="cuda")
    swih.match(cfg, plan.ws, 40, 40, 0, (10, 10, 9, 10), out,
               template_raw=torch.ones(4, dtype=torch.uint32, device="cuda"))
    torch.cuda.synchronize()
    assert out.item() == 7.0


# ---------------------------------------------------------------- Gaussian
@pytest.mark.parametrize("kind", GAUSS_KINDS)
def test_gaussian_scene512(scene512, kind):
    img, tc = scene512
    c = all_centres(512, 512, 31, 31)
    gauss_check(img, 16, 31, 31, c, tc, "gaussian(%d) 512x512 31x31" % kind, map_rect=(15, 15, 496, 496),
                kind=kind)


@pytest.mark.parametrize("kind", GAUSS_KINDS)
@pytest.mark.parametrize("HW,nb,wh", [((100, 77), 3, (5, 9)), ((65, 129), 16, (15, 21)),
                                      ((33, 33), 7, (33, 33)), ((20, 31), 5, (1, 1))])
def test_gaussian_ragged(HW, nb, wh, kind):
    H, W = HW
    w, h = wh
    img = synth.uniform_noise(H * 7 + W, H, W)
    c = all_centres(H, W, w, h)
    rx, ry = (w - 1) // 2, (h - 1) // 2
    gauss_check(img, nb, w, h, c, tuple(c[len(c) // 2]), "gaussian(%d) ragged %s %s" % (kind, HW, wh),
                map_rect=(rx, ry, W - 1 - rx, H - 1 - ry), kind=kind)


@pytest.mark.parametrize("kind", GAUSS_KINDS)
@pytest.mark.parametrize("K", [4, 6, 8])
def test_gaussian_other_series_lengths(K, kind):
    # K is a build parameter: longer series than the default (3), up to the
    # maximum (8), are just as exact
    H, W = 65, 129
    img = synth.uniform_noise(17 + K, H, W)
    c = all_centres(H, W, 15, 21)
    print("case: gaussian(%d) K=%d 65x129 16 bins 15x21" % (kind, K), flush=True)
    gauss_check(img, 16, 15, 21, c, tuple(c[len(c) // 3]), "gaussian(%d) K=%d" % (kind, K),
                map_rect=(7, 10, W - 8, H - 11), kind=kind, K=K)


@pytest.mark.parametrize("kind", GAUSS_KINDS)
def test_gaussian_windows_wider_than_a_block(kind):
    # wide windows on a map taller than two windows (several members per comb)
    H, W = 460, 420
    img = synth.smooth_noise(41, H, W)
    w, h = 161, 151
    c = synth.sample_centres(77, H, W, w, h, 2048)
    print("case: gaussian(%d) %dx%d window %dx%d" % (kind, H, W, w, h), flush=True)
    rx, ry = (w - 1) // 2, (h - 1) // 2
    gauss_check(img, 8, w, h, c, (W // 2, H // 2), "gaussian(%d) wide window" % kind,
                map_rect=(rx, ry, rx + 40, H - 1 - ry), kind=kind)


def test_gaussian_windows_wider_than_a_sweep_block():
    # windows wider than the twelve tiles of a sweep block: each block covers
    # its chunk's left-edge tiles and right-edge tiles apart (two tile ranges)
    H, W = 120, 1400
    img = synth.smooth_noise(43, H, W)
    w, h = 801, 15
    rx, ry = (w - 1) // 2, (h - 1) // 2
    c = synth.sample_centres(78, H, W, w, h, 256)
    print("case: gaussian %dx%d window %dx%d (two tile ranges per block)" % (H, W, w, h), flush=True)
    gauss_check(img, 6, w, h, c, (W // 2, H // 2), "gaussian two-range window",
                map_rect=(rx, ry, W - 1 - rx, ry + 2))


@pytest.mark.parametrize("w", [21, 31, 45, 63, 81])
def test_gaussian_multiscale_2048(w):
    # The multi-scale precision workload: 2048 x 2048 smooth noise, 32 bins,
    # the Gaussian at each of five scales (26 GB of planes per scale), template
    # at (1024, 1024).  Histograms at 4096 sampled centres (the valid region's
    # corners and edges included); the full valid map, computed as the
    # benchmark computes it (the comb sweep), checked on three whole rows of
    # centres (top, middle, bottom of the valid region) and at the sampled
    # centres, with the GPU's template and with the oracle's.
    H = W = 2048
    img = synth.smooth_noise(33, H, W)
    c = synth.sample_centres(100 + w, H, W, w, w, 4096)
    r = (w - 1) // 2
    print("case: gaussian 2048^2 32 bins scale %d" % w, flush=True)
    plan = Plan(swih.Config(32, swih.GAUSSIAN, [(w, w)]), H, W)
    plan.build(to_dev(img, torch))
    hist, _ = plan.query(0, to_dev(c, torch))
    t, _ = plan.query(0, to_dev(np.array([[1024, 1024]], np.int32), torch))
    pref = oracle.normalised(oracle.hist(img, 32, oracle.GAUSSIAN, w, w, c), oracle.GAUSSIAN, w, w)
    herr = float(np.abs(hist.cpu().numpy().astype(np.float64) - pref).max())
    _, tref = oracle.template(img, 32, oracle.GAUSSIAN, w, w, (1024, 1024))
    out = {"hist_err": herr}
    for name, tmpl in (("gpu_template", t[0].contiguous()),
                       ("oracle_template", to_dev(tref.astype(np.float32), torch))):
        m = plan.match(0, template=tmpl).cpu().numpy().astype(np.float64)
        assert m.shape == (H - w + 1, W - w + 1)
        errs = []
        for y in (r, 1024, H - 1 - r):
            mref = oracle.bc_map(img, 32, oracle.GAUSSIAN, w, w, tref, rect=(r, y, W - 1 - r, y))[0]
            errs.append(float(np.abs(m[y - r] - mref).max()))
        ms = oracle.bc_at(img, 32, oracle.GAUSSIAN, w, w, c, tref)
        errs.append(float(np.abs(m[c[:, 1] - r, c[:, 0] - r] - ms).max()))
        out[name] = errs
        assert max(errs) <= MAP_TOL, (w, name, errs)
    print("gaussian 2048 scale %d: hist err, map err on rows top/middle/bottom and sampled" % w, out,
          flush=True)
    assert herr <= GAUSS_TOL
    del plan
    torch.cuda.empty_cache()
