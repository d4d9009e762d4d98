"""GPU test of the continuous-batching server: every request's maps are the
same bit for bit as the one-request-at-a-time path, whatever micro-batch it
landed in and whichever requests shared it."""
import numpy as np
import pytest

from paper_1705_03524_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1705_03524_amd as swih  # noqa: E402
from paper_1705_03524_amd import serving  # noqa: E402


@pytest.mark.parametrize("direct", [True, False])
@pytest.mark.parametrize("kind", ["gaussian", "gaussian_sep", "exponential"])
def test_served_maps_equal_serial(kind, direct):
    # direct: micro-batches of one request use the single-unit calls
    print("case: serving 48 requests at 400 req/s vs serial, %s, direct singles %s" % (kind, direct),
          flush=True)
    cfg = swih.Config(16, kind, [(15, 15)])
    sizes = ((640, 480), (1280, 720))
    pool = serving.FramePool(sizes, lambda H, W: synth.smooth_noise(H + W, H, W))
    reqs = synth.serving_requests(3, 400.0, 48, nstreams=5, sizes=sizes)
    cont = serving.ContinuousServer(cfg, pool, budget=8 << 30, max_inflight=3, max_batch=6,
                                    direct_single=direct)
    got = cont.serve(reqs, keep_maps=True)
    torch.cuda.synchronize()
    ser = serving.SerialServer(cfg, pool, budget=8 << 30)
    ref = ser.serve(reqs, keep_maps=True)
    for a, b in zip(got, ref):
        assert len(a.host_maps) == 3
        for ma, mb in zip(a.host_maps, b.host_maps):
            assert torch.equal(ma, mb), a.id
    st = serving.latency_stats(got)
    assert st["requests"] == 48 and st["p99_ms"] >= st["p50_ms"] > 0
    # the served maps are likelihoods: within [0, 1], 1 near the stream's first target
    first = got[0].host_maps[1].numpy()
    assert first.max() <= 1.0 + 1e-6 and first.min() >= 0.0
    assert np.isclose(first.max(), 1.0, atol=1e-4)


@pytest.mark.parametrize("n,so,do", [(1, 0, 0), (15, 3, 3), (4099, 1, 7), (1 << 20, 16, 0),
                                     ((3 << 20) + 5, 5, 5)])
def test_copy_kernel_pinned_and_device(n, so, do):
    # every direction of the kernel copy, bit for bit, at any byte offset
    print("case: swih_copy n=%d src_off=%d dst_off=%d" % (n, so, do), flush=True)
    g = torch.Generator().manual_seed(n + so)
    src_h = torch.randint(0, 256, (n + 64,), dtype=torch.uint8, generator=g).pin_memory()
    dev = torch.zeros(n + 64, dtype=torch.uint8, device="cuda")
    back = torch.zeros(n + 64, dtype=torch.uint8).pin_memory()
    dev2 = torch.zeros(n + 64, dtype=torch.uint8, device="cuda")
    st = torch.cuda.Stream()
    swih.copy(dev[do:], src_h[so:], n, st)           # pinned host -> device
    swih.copy(dev2[so:], dev[do:], n, st)            # device -> device
    swih.copy(back[do:], dev2[so:], n, st)           # device -> pinned host
    st.synchronize()
    assert torch.equal(dev[do:do + n].cpu(), src_h[so:so + n])
    assert torch.equal(back[do:do + n], src_h[so:so + n])
    # bytes outside the range stay untouched
    assert int(back[:do].sum()) == 0 and int(back[do + n:].sum()) == 0
    assert int(dev[:do].sum().item()) == 0 and int(dev[do + n:].sum().item()) == 0


def test_copy_kernel_rejects_pageable_memory():
    print("case: swih_copy from pageable host memory", flush=True)
    src = torch.ones(4096, dtype=torch.uint8)  # not pinned
    dev = torch.zeros(4096, dtype=torch.uint8, device="cuda")
    with pytest.raises(swih.SwihError):
        swih.copy(dev, src, 4096)
    torch.cuda.synchronize()
    assert int(dev.sum().item()) == 0
