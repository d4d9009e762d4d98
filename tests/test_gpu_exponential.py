"""GPU parity of the exponential (Laplacian) kernel (SWIH_EXPONENTIAL).

Bar: normalised histograms within EXP_TOL = 2e-6 of the FP64 brute-force
oracle (the decomposition is exact; the bound on float rounding is derived in
tests/gpu_util.py), maps within MAP_TOL = 1e-5 of the oracle's map.  Cases:
* the 512 x 512 scene with every valid centre and the full map;
* ragged sizes, 1 to 256 bins, windows from 1 x 1 to the whole image;
* images far larger than exp(x / t) survives in any float format (2048^2 with
  3 x 3 windows, 8192^2), where only the rescaled planes stay bounded;
* several scales in one workspace, sub-rectangles, raw outputs rejected.
"""
import numpy as np
import pytest

import oracle
from paper_1705_03524_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1705_03524_amd as swih  # noqa: E402
from paper_1705_03524_amd.plan import Plan  # noqa: E402

from gpu_util import EXP_TOL, all_centres, gauss_check, to_dev  # noqa: E402

EXP = swih.EXPONENTIAL
OEXP = oracle.EXPONENTIAL


def check(img, nb, w, h, centres, tcentre, label, map_rect=None):
    return gauss_check(img, nb, w, h, centres, tcentre, label, map_rect=map_rect, kind=EXP,
                       okind=OEXP, tol=EXP_TOL)


def test_scene512():
    img, rects = synth.rect_scene(1, 512, 512)
    x0, y0, rw, rh, _ = rects[0]
    tc = (min(max(x0 + rw // 2, 15), 496), min(max(y0 + rh // 2, 15), 496))
    print("case: exponential 512x512 scene, 16 bins, 31x31, all windows", flush=True)
    check(img, 16, 31, 31, all_centres(512, 512, 31, 31), tc, "exp scene512",
          map_rect=(15, 15, 496, 496))


@pytest.mark.parametrize("HW,nb,wh", [
    ((100, 77), 3, (5, 9)),
    ((65, 129), 16, (15, 21)),
    ((130, 64), 256, (3, 3)),
    ((70, 200), 1, (7, 61)),
    ((33, 33), 7, (33, 33)),      # one window covering the whole image
    ((20, 31), 5, (1, 1)),        # single-pixel window
    ((1, 90), 4, (9, 1)),         # one row
    ((90, 1), 4, (1, 9)),         # one column
])
def test_ragged(HW, nb, wh):
    H, W = HW
    w, h = wh
    print("case: exponential ragged %dx%d bins %d window %dx%d" % (H, W, nb, w, h), flush=True)
    img = synth.uniform_noise(H * 13 + W, H, W)
    c = all_centres(H, W, w, h)
    rx, ry = (w - 1) // 2, (h - 1) // 2
    check(img, nb, w, h, c, tuple(c[len(c) // 2]), "exp ragged %s %s" % (HW, wh),
          map_rect=(rx, ry, W - 1 - rx, H - 1 - ry))


@pytest.mark.parametrize("w", [3, 31, 81, 201])
def test_large_image(w):
    # 2048^2: exp(x / t) with t = w / 4 leaves float range after ~90 t pixels
    H = W = 2048
    print("case: exponential 2048^2 32 bins %dx%d, sampled" % (w, w), flush=True)
    img = synth.smooth_noise(44, H, W)
    c = synth.sample_centres(300 + w, H, W, w, w, 4096)
    r = (w - 1) // 2
    c[0] = (r, r)
    c[1] = (W - 1 - r, H - 1 - r)
    c[2] = (r, H - 1 - r)
    c[3] = (W - 1 - r, r)
    check(img, 32, w, w, c, (1500, 700), "exp 2048 %d" % w,
          map_rect=(W - 1 - r - 70, H - 1 - r - 4, W - 1 - r, H - 1 - r))
    torch.cuda.empty_cache()


def test_max_side():
    H, W = 8192, 8192
    print("case: exponential 8192x8192, 4 bins, 61x61, sampled", flush=True)
    img = synth.uniform_noise(12, H, W)
    c = synth.sample_centres(13, H, W, 61, 61, 256)
    c[0] = (30, 30)
    c[1] = (W - 31, H - 31)
    check(img, 4, 61, 61, c, (4000, 5000), "exp 8192 61x61",
          map_rect=(W - 31 - 64, H - 31 - 2, W - 31, H - 31))
    torch.cuda.empty_cache()


def test_several_scales_and_rects():
    H, W = 260, 300
    img = synth.smooth_noise(6, H, W)
    scales = [(9, 9), (31, 15), (41, 61)]
    plan = Plan(swih.Config(8, EXP, scales), H, W)
    plan.build(to_dev(img, torch))
    for si, (w, h) in enumerate(scales):
        c = synth.sample_centres(si + 40, H, W, w, h, 300)
        got = plan.query(si, to_dev(c, torch))[0].cpu().numpy().astype(np.float64)
        ref = oracle.normalised(oracle.hist(img, 8, OEXP, w, h, c), OEXP, w, h)
        assert np.abs(got - ref).max() <= EXP_TOL, (w, h)
        # a map value depends on its centre only
        t = plan.query(si, to_dev(c[:1], torch))[0][0].contiguous()
        full = plan.match(si, template=t).cpu().numpy()
        x0, y0, x1, y1 = plan.valid_rect(si)
        for r in [(x0 + 3, y0 + 1, x1 - 5, y1), (x1, y1, x1, y1), (x0, y0 + 7, x0 + 64, y0 + 7)]:
            m = plan.match(si, template=t, rect=r).cpu().numpy()
            assert np.array_equal(m, full[r[1] - y0:r[3] - y0 + 1, r[0] - x0:r[2] - x0 + 1]), r


def test_raw_outputs_rejected():
    cfg = swih.Config(8, EXP, [(5, 5)])
    plan = Plan(cfg, 20, 20)
    plan.build(torch.zeros((20, 20), dtype=torch.uint8, device="cuda"))
    with pytest.raises(swih.SwihError):
        swih.query(cfg, plan.ws, 20, 20, 0, torch.zeros((1, 2), dtype=torch.int32, device="cuda"),
                   None, torch.empty((1, 8), dtype=torch.uint32, device="cuda"))
    with pytest.raises(swih.SwihError):
        swih.match(cfg, plan.ws, 20, 20, 0, (2, 2, 5, 5), torch.empty((4, 4), device="cuda"),
                   template_raw=torch.ones(8, dtype=torch.uint32, device="cuda"))


def test_constant_image_is_one_bin():
    img = np.full((70, 90), 200, np.uint8)
    plan = Plan(swih.Config(4, EXP, [(11, 7)]), 70, 90)
    plan.build(to_dev(img, torch))
    c = all_centres(70, 90, 11, 7)
    h = plan.query(0, to_dev(c, torch))[0].cpu().numpy()
    expect = np.zeros(4)
    expect[(200 * 4) // 256] = 1.0
    assert np.abs(h - expect).max() <= EXP_TOL
    m = plan.match(0, template=torch.tensor(expect, dtype=torch.float32, device="cuda")).cpu().numpy()
    assert np.abs(m - 1.0).max() <= 2e-6
