"""GPU tests of the one-launch batch (swih_run_batch).

* The persistent launch gives, bit for bit, what the stage launches give for
  the same table: every template histogram and every map, integer kernels and
  the 2-D Gaussian, uneven frames and crops with per-frame scales.
* The table can be launched again (the launch resets its counters), also after
  a launch whose waits were forced to give up, and inside a HIP graph.
* The failure path: with every wait forced to give up, the status word says so
  and the launch still ends.
"""
import pytest

from paper_1705_03524_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1705_03524_amd as swih  # noqa: E402

from gpu_util import to_dev  # noqa: E402
from test_gpu_batch import SCALES, SIZES, make_batch  # noqa: E402


def frames_for(kind):
    if kind == swih.GAUSSIAN:
        big = to_dev(synth.smooth_noise(91, 700, 900), torch)
        crops = [big[10:210, 20:300], big[300:420, 100:260], big[50:131, 400:690], big[500:560, 0:90],
                 big[100:612, 300:812]]
        scales = [[(21, 21), (31, 15)], [(15, 15)], [(9, 9), (25, 31), (41, 41)], [(11, 13)],
                  [(15, 15), (45, 45)]]
        return crops, scales
    imgs = [to_dev(synth.smooth_noise(60 + k, H, W), torch) for k, (H, W) in enumerate(SIZES)]
    scales = [[s for s in SCALES if s[0] <= W and s[1] <= H] for (H, W) in SIZES]
    return imgs, scales


def outputs(outs):
    res = {}
    for k, (c, rect, hist, raw, out) in outs.items():
        res[k] = (hist.clone(), None if raw is None else raw.clone(), out.clone())
    return res


def scrub(outs):
    for c, rect, hist, raw, out in outs.values():
        hist.fill_(-7.0)
        out.fill_(-7.0)
        if raw is not None:
            raw.fill_(12345)


def assert_same(a, b, label):
    for k in a:
        ha, ra, ma = a[k]
        hb, rb, mb = b[k]
        assert torch.equal(ha, hb), (label, k, "hist")
        if ra is not None:
            assert torch.equal(ra, rb), (label, k, "raw")
        assert torch.equal(ma, mb), (label, k, "map")


@pytest.mark.parametrize("kind,nb", [(swih.MANHATTAN, 16), (swih.MANHATTAN, 96), (swih.EUCLIDEAN, 16),
                                     (swih.UNIFORM, 32), (swih.GAUSSIAN, 16), (swih.GAUSSIAN, 32)])
def test_fused_equals_stage_launches(kind, nb):
    print("case: fused batch kind %d bins %d" % (kind, nb), flush=True)
    imgs, scales = frames_for(kind)
    integer = kind not in swih._swih.REAL_KINDS
    cfg = swih.Config(nb, kind, scales[0])
    b, outs = make_batch(cfg, imgs, scales, integer, list(range(len(imgs))))
    b.run()
    torch.cuda.synchronize()
    staged = outputs(outs)
    for rep in range(2):  # the second launch checks that the counters were reset
        scrub(outs)
        torch.cuda.synchronize()
        b.run_fused()
        torch.cuda.synchronize()
        assert b.fused_status() == 0
        assert_same(staged, outputs(outs), "rep %d" % rep)


def test_fused_graph_replay():
    print("case: fused batch captured in a graph", flush=True)
    imgs, scales = frames_for(swih.GAUSSIAN)
    cfg = swih.Config(16, swih.GAUSSIAN, scales[0])
    b, outs = make_batch(cfg, imgs, scales, False, list(range(len(imgs))))
    b.run()
    torch.cuda.synchronize()
    staged = outputs(outs)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        b.run_fused()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        b.run_fused()
    for rep in range(3):
        scrub(outs)
        junk = torch.randn(1 << 20, device="cuda").sum()  # other work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert junk.isfinite()
        assert b.fused_status() == 0
        assert_same(staged, outputs(outs), "replay %d" % rep)


def test_fused_failure_path_then_clean_run():
    # every wait forced to give up: the status says so, the launch ends, and the
    # next launch of the same table is exact again
    print("case: fused batch, waits forced to give up", flush=True)
    imgs, scales = frames_for(swih.MANHATTAN)
    cfg = swih.Config(16, swih.MANHATTAN, SCALES)
    b, outs = make_batch(cfg, imgs, scales, True, list(range(len(imgs))))
    b.run()
    torch.cuda.synchronize()
    staged = outputs(outs)
    b.run_fused(wait_ms=-1)
    torch.cuda.synchronize()
    assert b.fused_status() == 1
    scrub(outs)
    b.run_fused()
    torch.cuda.synchronize()
    assert b.fused_status() == 0
    assert_same(staged, outputs(outs), "after failure")


def test_fused_unsupported_kinds():
    print("case: fused batch refuses the separable and exponential kinds", flush=True)
    img = to_dev(synth.smooth_noise(5, 64, 80), torch)
    for kind in (swih.GAUSSIAN_SEP, swih.EXPONENTIAL):
        cfg = swih.Config(8, kind, [(9, 9)])
        b, _ = make_batch(cfg, [img], [[(9, 9)]], False, [0])
        with pytest.raises(swih.SwihError):
            b.run_fused()
