"""GPU test of swih_match_noalloc, the map entry point that allocates nothing:
its maps equal swih_match's bit for bit, over two calls in a row (the second
on a smaller rectangle), with a Gaussian plan whose bins are split into
groups (so the static scratch accumulator is used) and an integer kernel."""
import pytest

from paper_1705_03524_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1705_03524_amd as swih  # noqa: E402
from paper_1705_03524_amd.plan import Plan  # noqa: E402

from gpu_util import to_dev  # noqa: E402


@pytest.mark.parametrize("kind", [swih.GAUSSIAN, swih.MANHATTAN])
def test_noalloc_equals_match(kind):
    print("case: swih_match_noalloc vs swih_match, kind %d, two calls" % kind, flush=True)
    img = synth.smooth_noise(91, 512, 512)
    cfg = swih.Config(16, kind, [(31, 31)])
    integer = kind == swih.MANHATTAN
    for rect in ((15, 15, 496, 496), (40, 60, 300, 200)):   # full map, then a smaller one
        H, W = img.shape
        p = Plan(cfg, H, W)
        p.build(to_dev(img, torch))
        c = torch.tensor([[256, 256]], dtype=torch.int32, device="cuda")
        hist, raw = p.query(0, c)
        tmpl = None if integer else hist[0].contiguous()
        traw = raw[0].contiguous() if integer else None
        a = torch.full((rect[3] - rect[1] + 1, rect[2] - rect[0] + 1), -1.0, device="cuda")
        b = torch.full_like(a, -2.0)
        swih.match(cfg, p.ws, H, W, 0, rect, a, template=tmpl, template_raw=traw)
        swih.match_noalloc(cfg, p.ws, H, W, 0, rect, b, template=tmpl, template_raw=traw)
        torch.cuda.synchronize()
        assert torch.equal(a, b), rect
        assert float(a.max()) <= 1.0 + 1e-6 and float(a.min()) >= 0.0
        del p


def test_noalloc_rejects_oversized_rectangle():
    cfg = swih.Config(2, swih.GAUSSIAN, [(3, 3)])
    H, W = 2100, 2100          # 2098^2 centres > 2^22
    ws = torch.empty(16, dtype=torch.uint8, device="cuda")
    out = torch.empty(16, device="cuda")
    t = torch.ones(2, device="cuda") / 2
    with pytest.raises(swih.SwihError) as ei:
        swih.match_noalloc(cfg, ws, H, W, 0, (1, 1, H - 2, W - 2), out, template=t)
    assert ei.value.status == swih._swih.ERR_SCRATCH
