"""GPU tests of the batched form (swih_batch_plan / swih_*_batch).

* A batch of uneven frames gives, for every frame, exactly (bit for bit) what
  the single-frame calls give, and those match the oracle (spot checks).
* Mix invariance: a frame's histograms and map are identical alone and inside
  batches with other frames in any order.
* The whole batch captured once in a HIP graph replays to the eager results,
  with other GPU work between replays.
"""
import numpy as np
import pytest

import oracle
from paper_1705_03524_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1705_03524_amd as swih  # noqa: E402
from paper_1705_03524_amd.batch import Batch  # noqa: E402
from paper_1705_03524_amd.plan import Plan  # noqa: E402

from gpu_util import to_dev  # noqa: E402

SIZES = [(97, 131), (256, 300), (64, 64), (300, 200), (513, 127), (40, 50)]
SCALES = [(15, 15), (9, 21), (31, 31)]


def frame_jobs(H, W, scales, seed, nb, integer):
    """One ROI per frame: template query at its centre, map over its search box."""
    g = synth.rng(seed)
    qs, ms = [], []
    for si, (w, h) in enumerate(scales):
        rx, ry = (w - 1) // 2, (h - 1) // 2
        if W - 1 - rx < rx or H - 1 - ry < ry:
            continue
        cx = int(g.integers(rx, W - rx))
        cy = int(g.integers(ry, H - ry))
        x0, x1 = max(rx, cx - 2 * w), min(W - 1 - rx, cx + 2 * w)
        y0, y1 = max(ry, cy - 2 * h), min(H - 1 - ry, cy + 2 * h)
        qs.append((si, (cx, cy)))
        ms.append((si, (x0, y0, x1, y1)))
    return qs, ms


def make_batch(cfg, imgs, scales_per_frame, integer, order):
    frames, queries, matches, outs = [], [], [], {}
    for slot, fi in enumerate(order):
        img = imgs[fi]
        H, W = img.shape
        frames.append({"img": img, "scales": scales_per_frame[fi]})
        qs, ms = frame_jobs(H, W, scales_per_frame[fi], 1000 + fi, cfg.nbins, integer)
        for (si, c), (_, rect) in zip(qs, ms):
            cen = torch.tensor([c], dtype=torch.int32, device="cuda")
            hist = torch.empty((1, cfg.nbins), dtype=torch.float32, device="cuda")
            raw = torch.empty((1, cfg.nbins), dtype=torch.uint32, device="cuda") if integer else None
            queries.append({"frame": slot, "scale_idx": si, "centres": cen, "hist": hist, "hist_raw": raw})
            x0, y0, x1, y1 = rect
            out = torch.empty((y1 - y0 + 1, x1 - x0 + 1), dtype=torch.float32, device="cuda")
            m = {"frame": slot, "scale_idx": si, "rect": rect, "out": out}
            if integer:
                m["template_raw"] = raw[0]
            else:
                m["template"] = hist[0]
            matches.append(m)
            outs[(fi, si)] = (c, rect, hist, raw, out)
    return Batch(cfg, frames, queries, matches), outs


def single(cfg, img, scales, si, c, rect, integer):
    fc = swih.Config(cfg.nbins, cfg.kernel, scales, cfg.gauss_terms)
    p = Plan(fc, img.shape[0], img.shape[1])
    p.build(img)
    hist, raw = p.query(si, torch.tensor([c], dtype=torch.int32, device="cuda"))
    if integer:
        out = p.match(si, template_raw=raw[0].contiguous(), rect=rect)
    else:
        out = p.match(si, template=hist[0].contiguous(), rect=rect)
    return hist, raw, out


# 16 bins: the histogram aggregate in the batch; 96: the per-bin aggregate
@pytest.mark.parametrize("nb", [16, 96])
@pytest.mark.parametrize("kind", [swih.MANHATTAN, swih.EUCLIDEAN])
def test_batch_equals_single_integer(kind, nb):
    print("case: batch integer kind %d bins %d" % (kind, nb), flush=True)
    cfg = swih.Config(nb, kind, SCALES)
    imgs = [to_dev(synth.smooth_noise(10 + k, H, W), torch) for k, (H, W) in enumerate(SIZES)]
    scales = [[s for s in SCALES if s[0] <= W and s[1] <= H] for (H, W) in SIZES]
    b, outs = make_batch(cfg, imgs, scales, True, list(range(len(imgs))))
    b.run()
    torch.cuda.synchronize()
    checked = 0
    for (fi, si), (c, rect, hist, raw, out) in outs.items():
        sh, sr, so = single(cfg, imgs[fi], scales[fi], si, c, rect, True)
        assert torch.equal(raw, sr) and torch.equal(out, so), (fi, si)
        if checked < 4:  # oracle spot check
            img = imgs[fi].cpu().numpy()
            w, h = scales[fi][si]
            tref, _ = oracle.template(img, nb, kind, w, h, c)
            assert np.array_equal(raw.cpu().numpy()[0].astype(np.int64), tref)
            mref = oracle.bc_map(img, nb, kind, w, h, tref, rect=rect)
            assert np.array_equal(out.cpu().numpy(), mref.astype(np.float32))
            checked += 1


# exponential: 16 bins take the histogram aggregate, 40 the per-bin one
@pytest.mark.parametrize("nb", [16, 40])
@pytest.mark.parametrize("kind", [swih.GAUSSIAN, swih.GAUSSIAN_SEP, swih.EXPONENTIAL])
def test_batch_equals_single_gaussian_crops(kind, nb):
    print("case: batch real-valued kind %d bins %d: crops with per-frame scales" % (kind, nb), flush=True)
    big = to_dev(synth.smooth_noise(77, 600, 700), torch)
    crops = [big[10:210, 20:300], big[300:420, 100:260], big[50:131, 400:690], big[500:560, 0:90]]
    scales = [[(21, 21), (31, 15)], [(15, 15)], [(9, 9), (25, 31), (41, 41)], [(11, 13)]]
    cfg = swih.Config(nb, kind, [(15, 15)])
    b, outs = make_batch(cfg, crops, scales, False, list(range(len(crops))))
    b.run()
    torch.cuda.synchronize()
    for (fi, si), (c, rect, hist, raw, out) in outs.items():
        sh, _, so = single(cfg, crops[fi], scales[fi], si, c, rect, False)
        assert torch.equal(hist, sh) and torch.equal(out, so), (fi, si)
    # oracle spot check on one crop
    fi, si = 2, 1
    c, rect, hist, _, out = outs[(fi, si)]
    img = crops[fi].cpu().numpy()
    w, h = scales[fi][si]
    ok = oracle.EXPONENTIAL if kind == swih.EXPONENTIAL else oracle.GAUSSIAN
    _, tp = oracle.template(img, nb, ok, w, h, c)
    assert np.abs(hist.cpu().numpy()[0] - tp).max() <= 1e-5


def test_mix_invariance():
    print("case: mix invariance", flush=True)
    cfg = swih.Config(16, swih.MANHATTAN, SCALES)
    imgs = [to_dev(synth.smooth_noise(30 + k, H, W), torch) for k, (H, W) in enumerate(SIZES)]
    scales = [[s for s in SCALES if s[0] <= W and s[1] <= H] for (H, W) in SIZES]
    results = []
    for order in ([1], [0, 1, 2, 3, 4, 5], [5, 3, 1, 0], [1, 1]):
        b, outs = make_batch(cfg, imgs, scales, True, order)
        b.run()
        torch.cuda.synchronize()
        results.append({k: (v[3].clone(), v[4].clone()) for k, v in outs.items() if k[0] == 1})
    for r in results[1:]:
        for k in results[0]:
            assert torch.equal(results[0][k][0], r[k][0]) and torch.equal(results[0][k][1], r[k][1])
    # Gaussian too
    gcfg = swih.Config(16, swih.GAUSSIAN, [(15, 15), (21, 21)])
    gres = []
    for order in ([2], [0, 2, 4], [4, 2]):
        b, outs = make_batch(gcfg, imgs, [[(15, 15), (21, 21)]] * len(imgs), False, order)
        b.run()
        torch.cuda.synchronize()
        gres.append({k: (v[2].clone(), v[4].clone()) for k, v in outs.items() if k[0] == 2})
    for r in gres[1:]:
        for k in gres[0]:
            assert torch.equal(gres[0][k][0], r[k][0]) and torch.equal(gres[0][k][1], r[k][1])


@pytest.mark.parametrize("kind", [swih.MANHATTAN, swih.GAUSSIAN, swih.GAUSSIAN_SEP, swih.EXPONENTIAL])
def test_graph_replay(kind):
    print("case: graph replay kind %d" % kind, flush=True)
    cfg = swih.Config(16, kind, SCALES)
    imgs = [to_dev(synth.smooth_noise(50 + k, H, W), torch) for k, (H, W) in enumerate(SIZES)]
    scales = [[s for s in SCALES if s[0] <= W and s[1] <= H] for (H, W) in SIZES]
    integer = kind not in swih._swih.REAL_KINDS
    b, outs = make_batch(cfg, imgs, scales, integer, list(range(len(imgs))))
    b.run()
    torch.cuda.synchronize()
    eager = {k: v[4].clone() for k, v in outs.items()}
    b.capture()
    for rep in range(3):
        for k, v in outs.items():
            v[4].fill_(-1.0)
        junk = torch.randn(1 << 20, device="cuda").sum()  # other work between replays
        torch.cuda.synchronize()
        b.replay()
        torch.cuda.synchronize()
        assert junk.isfinite()
        for k, v in outs.items():
            assert torch.equal(v[4], eager[k]), (rep, k)


def test_batch_rejects_bad_descriptors():
    cfg = swih.Config(8, swih.MANHATTAN, [(5, 5)])
    img = torch.zeros((20, 20), dtype=torch.uint8, device="cuda")
    with pytest.raises(swih.SwihError):
        Batch(cfg, [{"img": img}], [], [{"frame": 1, "rect": (2, 2, 5, 5), "out": img,
                                          "template_raw": img}])
    with pytest.raises(swih.SwihError):   # window outside the frame
        Batch(cfg, [{"img": img}], [], [{"frame": 0, "rect": (1, 2, 5, 5), "out": img,
                                          "template_raw": img}])
