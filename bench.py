"""Benchmark of the SWIH hot path on one MI355X.

Headline workload (the multi-scale configuration, the largest that the paper's
title case puts on one GPU): a 2048 x 2048 uint8 smooth-noise image (uniform
noise blurred with sigma 3, stretched to 0..255), 32 bins, the Gaussian kernel
(sigma = w/4, K = 3 cosine series, 49 weight terms) at the five window scales
21, 31, 45, 63 and 81.  One step = for every scale: build the weighted integral
histograms of the scale (26 GB of planes, one workspace reused across the
scales), query the template histogram at (1024, 1024) and compute the
Bhattacharyya likelihood map of every valid centre (20.0 M windows per step).
The image is resident in HBM before the timed region starts.

Reported beside it (same JSON line): the 512 x 512 single-frame step with three
kernels, the 2048 x 2048 builds of the Manhattan, exponential and Gaussian
kernels, the batched workload (64 uneven frames, per-frame loop against one
batch), the measured write-only and copy ceilings of the machine's HBM, and the CPU
oracle on sampled centres of the headline workload.

Prints one JSON line (metric = weighted local histograms per second).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

HBM_PEAK_GBS = 8000.0
METRIC = "weighted local histograms/sec + IH-build HBM GB/s; served p50/p99 latency"
H = W = 512
NBINS = 16
WIN = 31
KERNELS = ("manhattan", "euclidean", "gaussian")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="target CPU time of the oracle sample")
    ap.add_argument("--workload", choices=("multiscale", "frame", "batch", "serve", "sweep", "track",
                                           "builds", "ceilings"),
                    default="multiscale",
                    help="multiscale: 2048x2048, 32 bins, Gaussian at 5 scales (default); frame: the "
                         "512x512 single-frame path; batch: 64 uneven frames with 1-8 targets x 3 "
                         "scales, batched vs per-frame; serve: Poisson tracking requests, continuous "
                         "batching vs one at a time; ceilings: HBM write-only and copy rates")
    ap.add_argument("--rates", default="50,100,200,500,1000,2000",
                    help="serve workload: request rates (req/s) to sweep")
    ap.add_argument("--seconds", type=float, default=1.0,
                    help="serve workload: arrival span per rate")
    ap.add_argument("--serve-trace", default=None,
                    help="serve workload: append each rate's per-request host timeline "
                         "(continuous server) to this JSONL file")
    ap.add_argument("--gaussian", choices=("2d", "separable"), default="2d",
                    help="batch / serve workloads: the Gaussian as 2-D planes (49 weight terms) "
                         "or in separable form")
    ap.add_argument("--budget-gb", type=float, default=64.0,
                    help="batch workload: workspace budget of one Gaussian sub-batch")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the measurements reported beside the step (separable Gaussian, exponential, "
                         "2048x2048 builds), so a profile of the run covers the step's launches only")
    ap.add_argument("--streams", type=int, choices=(1, 3), default=3,
                    help="frame workload: run the three kernels' pipelines (each build -> query -> "
                         "map in order) on 3 streams forked and joined inside the step's graph, or "
                         "all on one stream")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a 1 GiB device-to-device copy (known bytes) so HBM "
                         "counters of a profiling run can be scaled")
    return ap.parse_args()


def scene():
    from paper_1705_03524_amd import synth
    img, rects = synth.rect_scene(1, H, W)
    x0, y0, rw, rh, _ = rects[0]
    r = (WIN - 1) // 2
    tc = (min(max(x0 + rw // 2, r), W - 1 - r), min(max(y0 + rh // 2, r), H - 1 - r))
    return img, tc


def synth_smooth(n):
    from paper_1705_03524_amd import synth
    return synth.smooth_noise(33, n, n)


def cpu_baseline(img, tc, budget_s):
    """The oracle (brute force, OpenMP over centres) on a bounded sample: rows of
    centres of the same map, all three kernels, until ~budget_s of wall time
    (wrapping round to the first row if the whole map finishes first)."""
    import oracle
    kinds = {"manhattan": oracle.MANHATTAN, "euclidean": oracle.EUCLIDEAN, "gaussian": oracle.GAUSSIAN}
    r = (WIN - 1) // 2
    templ = {}
    for k, kind in kinds.items():
        raw, p = oracle.template(img, NBINS, kind, WIN, WIN, tc)
        templ[k] = raw if kind != oracle.GAUSSIAN else p
    rows = 0
    windows = 0
    t0 = time.perf_counter()
    y = r
    while time.perf_counter() - t0 < budget_s:
        for k, kind in kinds.items():
            oracle.bc_map(img, NBINS, kind, WIN, WIN, templ[k], rect=(r, y, W - 1 - r, y))
            windows += W - 2 * r
        rows += 1
        y = y + 1 if y < H - 1 - r else r
    dt = time.perf_counter() - t0
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": windows / dt, "unit": "windows/s", "cores": threads, "kind": "oracle",
            "sample": "%d centre rows x 3 kernels (%d windows) of the 512x512 map, cycling through "
                      "its %d rows, %.1f s" % (rows, windows, H - 2 * r, dt)}


PROFILE_COUNTERS = os.path.join(HERE, "profiles", "swih_512_scene_hbm_counters.md")
PROFILE_COUNTERS_MS = os.path.join(HERE, "profiles", "swih_2048_multiscale_hbm_counters.md")

# The multi-scale workload: 2048 x 2048 smooth noise, 32 bins, Gaussian at five
# scales, template at the image centre.
MS_SIDE = 2048
MS_BINS = 32
MS_SCALES = (21, 31, 45, 63, 81)
MS_TEMPLATE = (1024, 1024)


def host_info():
    """Core count and CPU model of the host the oracle runs on."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "cpu_model": model,
            "omp_num_threads_env": os.environ.get("OMP_NUM_THREADS")}


def cpu_baseline_multiscale(img, nsample=65536):
    """The oracle (brute force per window, FP64, OpenMP over centres) on
    ``nsample`` seeded centres per scale of the multi-scale workload (the valid
    region's corners and edges included), on all the threads it runs with and
    on one; windows/s is extrapolated from the sample to the full maps."""
    import oracle
    from paper_1705_03524_amd import synth
    threads = oracle.threads()
    samples, tmpl = {}, {}
    for w in MS_SCALES:
        samples[w] = synth.sample_centres(500 + w, MS_SIDE, MS_SIDE, w, w, nsample)
        tmpl[w] = oracle.template(img, MS_BINS, oracle.GAUSSIAN, w, w, MS_TEMPLATE)[1]
    out = {}
    for label, n in (("all", threads), ("one", 1)):
        oracle.set_threads(n)
        oracle.bc_at(img, MS_BINS, oracle.GAUSSIAN, 21, 21, samples[21][:64], tmpl[21])  # thread pool up
        t0 = time.perf_counter()
        for w in MS_SCALES:
            oracle.bc_at(img, MS_BINS, oracle.GAUSSIAN, w, w, samples[w], tmpl[w])
        out[label] = time.perf_counter() - t0
    oracle.set_threads(threads)
    nwin = nsample * len(MS_SCALES)
    per_step = sum((MS_SIDE - w + 1) ** 2 for w in MS_SCALES)
    return {"value": nwin / out["all"], "unit": "windows/s", "cores": threads, "kind": "oracle",
            "sample": "%d seeded centres per scale (valid-region corners and edges included) x %d scales "
                      "of the 2048x2048 multi-scale workload, brute force per window in FP64; "
                      "windows/s extrapolated from the sample to the full maps (%.1f s on %d threads, "
                      "%.1f s on 1)" % (nsample, len(MS_SCALES), out["all"], threads, out["one"]),
            "extrapolated": True,
            "one_core": {"value": nwin / out["one"], "unit": "windows/s", "cores": 1},
            "full_step_s_extrapolated": per_step / (nwin / out["all"]),
            "host": host_info()}


GAUSS_PLANES = 5  # corner-contracted planes per bin: four corners and the count


def gauss_side_bytes(K, B, H, W, TY=64):
    """Bytes of a Gaussian plane set besides its planes: the row carries (2 (2K+1) + 1
    FP64 values per bin, tile column of 64 pixels and row) and the band-closing rows
    (2 (2K+1) floats per bin and column at every multiple of TY below H)."""
    nt = 2 * K + 1
    return 8 * (2 * nt + 1) * B * ((W + 63) // 64) * (H + 1) + 4 * 2 * nt * B * W * ((H - 1) // TY)


def kernel_source_hash():
    import hashlib
    h = hashlib.sha1()
    for f in ("swih_build.hip", "swih_build_bodies.h", "swih_query.hip", "swih_query_bodies.h",
              "swih_layout.h", "wave64.h"):
        with open(os.path.join(HERE, "paper_1705_03524_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(prefixes, unit_prefix, path=PROFILE_COUNTERS):
    """HBM bytes per launch of a phase from a committed counter summary
    (scaled FETCH_SIZE + WRITE_SIZE): the bytes of every kernel whose name
    starts with one of `prefixes`, over all its dispatches, divided by the
    dispatches of the phase's main kernel (`unit_prefix`).  None if the
    summary is missing or was taken on different kernel sources."""
    try:
        txt = open(path).read()
    except OSError:
        return None
    if kernel_source_hash() not in txt:
        return None
    total, units = 0.0, 0
    for line in txt.splitlines():
        cells = [c.strip() for c in line.strip().strip("|").split("|")]
        if len(cells) != 6 or not cells[1].isdigit():
            continue
        n = int(cells[1])
        if any(cells[0].startswith(p) for p in prefixes):
            total += (float(cells[4]) + float(cells[5])) * 1e6 * n
        if cells[0].startswith(unit_prefix):
            units += n
    return total / units if units else None


def copy_calibration():
    """One 1 GiB device-to-device copy (1 GiB read, 1 GiB written), so that the
    HBM counters of a profiling run can be scaled to bytes."""
    import torch
    src = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


def capture_graph(fn):
    """Capture fn's launches (on the current stream) as one HIP graph, after one
    eager run on a side stream."""
    import torch
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        fn()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        fn()
    torch.cuda.synchronize()
    return g


def time_launches(fn, rep, replays=3):
    """Average duration (ms) of one launch of fn: rep launches captured back to
    back in one graph, replayed between HIP events on the launch stream."""
    import torch
    g = capture_graph(lambda: [fn() for _ in range(rep)])
    g.replay()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(replays):
        g.replay()
    b.record()
    torch.cuda.synchronize()
    del g
    return a.elapsed_time(b) / (replays * rep)


def ceilings():
    """Measured HBM ceilings of the box: a write-only fill and a device copy of
    4 GiB buffers (torch's own kernels), bytes moved per second."""
    import torch
    n = 4 << 30
    x = torch.empty(n, dtype=torch.uint8, device="cuda")
    y = torch.empty_like(x)
    x.fill_(1)
    y.copy_(x)
    torch.cuda.synchronize()
    fill_ms = time_launches(lambda: x.fill_(3), 5)
    copy_ms = time_launches(lambda: y.copy_(x), 5)
    del x, y
    torch.cuda.empty_cache()
    return {"write_only_gbs": n / (fill_ms / 1e3) / 1e9, "copy_gbs": 2 * n / (copy_ms / 1e3) / 1e9,
            "copy_bytes_counted": "read + write", "buffer_bytes": n,
            "kernels": "torch fill_ and copy_ on uint8 tensors",
            "write_only_frac_of_peak": n / (fill_ms / 1e3) / 1e9 / HBM_PEAK_GBS,
            "copy_frac_of_peak": 2 * n / (copy_ms / 1e3) / 1e9 / HBM_PEAK_GBS}


def run_multiscale(args):
    """The headline: 2048 x 2048 smooth noise, 32 bins, Gaussian at scales 21,
    31, 45, 63, 81; per scale build + template query + full valid map, one
    workspace reused across the scales; returns the JSON line (a dict)."""
    import torch
    import paper_1705_03524_amd as swih
    from paper_1705_03524_amd.plan import Plan

    N, B = MS_SIDE, MS_BINS
    img = synth_smooth(N)
    d_img = torch.from_numpy(img).cuda()
    d_tc = torch.tensor([MS_TEMPLATE], dtype=torch.int32, device="cuda")
    cfgs = [swih.Config(B, swih.GAUSSIAN, [(w, w)]) for w in MS_SCALES]
    nbytes = max(swih.workspace_bytes(c, N, N) for c in cfgs)
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    plans = [Plan(c, N, N, ws=ws) for c in cfgs]
    maps = [torch.empty((N - w + 1, N - w + 1), dtype=torch.float32, device="cuda") for w in MS_SCALES]
    tmpl = [torch.empty((1, B), dtype=torch.float32, device="cuda") for _ in MS_SCALES]
    PHASES = ("carries", "planes", "query", "match")

    def phase(si, name):
        p = plans[si]
        if name in ("carries", "planes"):
            swih.build_phase(p.cfg, d_img, p.ws, name, 0)
        elif name == "query":
            swih.query(p.cfg, p.ws, N, N, 0, d_tc, tmpl[si], None)
        else:
            swih.match(p.cfg, p.ws, N, N, 0, p.valid_rect(0), maps[si], template=tmpl[si][0])

    def step():
        for si in range(len(MS_SCALES)):
            for ph in PHASES:
                phase(si, ph)

    if args.copy_calibration:
        copy_calibration()
    for _ in range(max(1, args.warmup)):
        step()
    torch.cuda.synchronize()
    eager = [m.clone() for m in maps]
    g_step = capture_graph(step)
    for m in maps:
        m.fill_(-1.0)
    g_step.replay()
    torch.cuda.synchronize()
    for si, m in enumerate(maps):
        if not torch.equal(m, eager[si]):
            raise RuntimeError("graph replay of scale %d differs from the eager step" % MS_SCALES[si])
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0.record()
    for _ in range(args.steps):
        g_step.replay()
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / args.steps
    del g_step
    # Per-launch durations, scale by scale in pipeline order (each phase leaves
    # the workspace as the next one needs it).
    reps = {"carries": 10, "planes": 3, "query": 10, "match": 3}
    per = {}
    for si, w in enumerate(MS_SCALES):
        for ph in PHASES:
            per["%s_%d" % (ph, w)] = time_launches(lambda: phase(si, ph), reps[ph])
    nwin = [(N - w + 1) ** 2 for w in MS_SCALES]
    T = GAUSS_PLANES
    plane_bytes = 4 * T * B * (N + 1) * (N + 1)
    rc_bytes = gauss_side_bytes(cfgs[0].K, B, N, N)
    nsc = len(MS_SCALES)
    kernels = {
        "build": {"kernel": "emit_gauss (Gaussian plane build, %d planes x %d bins + row carries, "
                            "2048x2048; average over the 5 scales)" % (T, B),
                  "alg": N * N + plane_bytes + rc_bytes,
                  "ms": sum(per["planes_%d" % w] for w in MS_SCALES) / nsc,
                  "prefixes": ("emit_gauss",), "unit": "emit_gauss"},
        "match": {"kernel": "k_sweep + match_gauss_fin (Gaussian dense likelihood map, "
                            "every valid centre; average over the 5 scales)",
                  "alg": plane_bytes + rc_bytes + 4 * sum(nwin) / nsc,
                  "ms": sum(per["match_%d" % w] for w in MS_SCALES) / nsc,
                  "prefixes": ("k_sweep", "match_gauss_fin"), "unit": "k_sweep"},
    }

    def roof(k):
        achieved = k["alg"] / (k["ms"] / 1e3) / 1e9
        return {"bound": "hbm", "kernel": k["kernel"], "achieved": achieved, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                "traffic": measured_traffic(k["prefixes"], k["unit"], PROFILE_COUNTERS_MS),
                "alg_bytes_per_launch": k["alg"], "avg_launch_ms": k["ms"]}

    dominant = max(kernels, key=lambda n: kernels[n]["ms"])
    other = "build" if dominant == "match" else "match"
    per_scale = {}
    for si, w in enumerate(MS_SCALES):
        build_ms = per["carries_%d" % w] + per["planes_%d" % w]
        per_scale[str(w)] = {
            "windows": nwin[si],
            "ms": build_ms + per["query_%d" % w] + per["match_%d" % w],
            "ih_build_gbs": (N * N + plane_bytes + rc_bytes) / (build_ms / 1e3) / 1e9,
            "ih_build_frac": (N * N + plane_bytes + rc_bytes) / (build_ms / 1e3) / 1e9 / HBM_PEAK_GBS,
            "map_gbs": (plane_bytes + 4 * nwin[si]) / (per["match_%d" % w] / 1e3) / 1e9}
    line = {
        "metric": METRIC,
        "value": sum(nwin) / (ms / 1e3),
        "unit": "windows/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "multi-scale: 2048x2048 smooth noise (seed 33), 32 bins, Gaussian kernel "
                               "(sigma = w/4, K=3 cosine series, 49 weight terms) at scales 21,31,45,63,81; "
                               "per scale: IH build + template query at (1024,1024) + Bhattacharyya map of "
                               "every valid centre; one 27 GB workspace reused across scales",
                   "windows_per_step": sum(nwin), "global_batch": 1, "seq_len": None,
                   "parallelism": "none"},
        "roofline": roof(kernels[dominant]),
        "roofline_" + other: roof(kernels[other]),
        "detail_ms": per,
        "per_scale": per_scale,
    }
    del plans, ws, maps
    torch.cuda.empty_cache()
    return line, img


def bench_batch(args):
    print(json.dumps(run_batch(args)), flush=True)


def run_batch(args):
    """64 uneven frames (256..1920 x 256..1080), 1-8 targets of side 16..128,
    3 scales each, search region 3s x 3s, 16 bins; Manhattan (one build per
    frame) and Gaussian K=3 (one build per target-scale search crop).  Times
    the plain per-frame loop of single calls, the batched form, and the batched
    form replayed from one HIP graph; checks batched == per-frame bit for bit."""
    import torch
    import paper_1705_03524_amd as swih
    from paper_1705_03524_amd import workloads as WL

    frames = WL.batch_config_frames(4, 64)
    out = {}
    total_windows = 0
    total_ms = {"per_frame": 0.0, "batched": 0.0, "graph": 0.0, "fused": 0.0}
    gname = "gaussian_sep" if args.gaussian == "separable" else "gaussian"
    for name in ("manhattan", gname):
        cfg = swih.Config(16, name, [(15, 15)])
        units = WL.tracking_units(cfg, frames)
        budget = int(args.budget_gb * 2**30)
        per = WL.PerFrameRunner(cfg, units, budget)
        bat = WL.BatchedRunner(cfg, units, budget)
        # correctness: batched results equal the per-frame ones bit for bit
        per.run()
        torch.cuda.synchronize()
        ref = [j.out.clone() for u in units for j in u.jobs]
        for u in units:
            for j in u.jobs:
                j.out.fill_(-1)
        bat.run()
        torch.cuda.synchronize()
        same = all(torch.equal(a, j.out) for a, j in zip(ref, (j for u in units for j in u.jobs)))
        # the one-launch form (one persistent launch per sub-batch)
        for u in units:
            for j in u.jobs:
                j.out.fill_(-1)
        bat.run_fused()
        torch.cuda.synchronize()
        same_fused = bat.fused_status() == 0 and all(
            torch.equal(a, j.out) for a, j in zip(ref, (j for u in units for j in u.jobs)))
        bat.capture()

        def timed(fn, steps):
            for _ in range(max(1, args.warmup // 2)):
                fn()
            torch.cuda.synchronize()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            for _ in range(steps):
                fn()
            b.record()
            torch.cuda.synchronize()
            return a.elapsed_time(b) / steps

        steps = max(1, args.steps // 4)
        t_per = timed(per.run, steps)
        t_bat = timed(bat.run, steps)
        t_gra = timed(bat.replay, steps)
        t_fus = timed(bat.run_fused, steps)
        # the same batch with scan tiles picked by the autotuner per unit size class
        from paper_1705_03524_amd.autotune import Autotuner
        tuner = Autotuner()  # cache: $SWIH_AUTOTUNE_CACHE, else ~/.cache/swih_autotune.json
        chosen = WL.tune_units(cfg, units, tuner)
        tun = WL.BatchedRunner(cfg, units, budget)
        for u in units:
            for j in u.jobs:
                j.out.fill_(-1)
        tun.run()
        torch.cuda.synchronize()
        tdiff = max(float((a - j.out).abs().max()) for a, j in zip(ref, (j for u in units for j in u.jobs)))
        tun.capture()
        t_tun = timed(tun.run, steps)
        t_tgr = timed(tun.replay, steps)
        nw = WL.total_windows(units)
        total_windows += nw
        total_ms["per_frame"] += t_per
        total_ms["batched"] += t_bat
        total_ms["graph"] += t_gra
        total_ms["fused"] += t_fus
        out[name] = {"units": len(units), "jobs": sum(len(u.jobs) for u in units),
                     "sub_batches": bat.nbatches, "windows": nw,
                     "plane_gb": WL.plane_bytes(cfg, units) / 1e9,
                     "ms_per_frame_loop": t_per, "ms_batched": t_bat, "ms_graph": t_gra,
                     "windows_per_s_graph": nw / (t_gra / 1e3), "batched_equals_per_frame": same,
                     "ms_fused": t_fus, "windows_per_s_fused": nw / (t_fus / 1e3),
                     "fused_equals_per_frame": same_fused,
                     "autotuned": {"band_rows_by_size_class": {"%dx%d" % (c[1], c[0]): r
                                                               for c, r in sorted(chosen.items())},
                                   "ms_batched": t_tun, "ms_graph": t_tgr,
                                   "max_abs_map_diff_vs_default_tiles": tdiff}}
        total_ms["tuned"] = total_ms.get("tuned", 0.0) + min(t_tun, t_tgr)
        del per, bat, tun, units
        torch.cuda.empty_cache()
    best = min(total_ms["batched"], total_ms["graph"])
    line = {
        "metric": METRIC, "value": total_windows / (best / 1e3), "unit": "windows/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": best,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32+f32",
        "data": "synthetic",
        "config": {"workload": "batch: 64 uneven frames 256..1920 x 256..1080, 1-8 targets side "
                               "16..128 x 3 scales, search 3s x 3s, 16 bins, Manhattan + Gaussian K=3 "
                               "(%s)" % ("separable" if args.gaussian == "separable" else "2-D planes"),
                   "global_batch": 64, "seq_len": None, "parallelism": "none"},
        "per_frame_windows_per_s": total_windows / (total_ms["per_frame"] / 1e3),
        "speedup_vs_per_frame": total_ms["per_frame"] / best,
        "fused_windows_per_s": total_windows / (total_ms["fused"] / 1e3),
        "fused_speedup_vs_per_frame": total_ms["per_frame"] / total_ms["fused"],
        "autotuned_windows_per_s": total_windows / (total_ms["tuned"] / 1e3),
        "detail": out,
    }
    return line


def bench_serve(args):
    """Poisson tracking requests from 16 streams (frames 640x480..4096x2160,
    target 24..96 px, 3 scales, search 2-4x target, 16 bins, Gaussian K=3);
    continuous batching (3 in-flight micro-batches, 24 GiB workspace each) vs
    one request at a time, swept over arrival rates."""
    import torch
    import paper_1705_03524_amd as swih
    from paper_1705_03524_amd import serving, synth

    cfg = swih.Config(16, "gaussian_sep" if args.gaussian == "separable" else "gaussian", [(15, 15)])
    pool = serving.FramePool(synth.FRAME_SIZES, lambda H, W: synth.smooth_noise(H * 7 + W, H, W))
    cont = serving.ContinuousServer(cfg, pool, budget=24 << 30, max_inflight=3)
    cont.trace = bool(args.serve_trace)
    ser = serving.SerialServer(cfg, pool, budget=8 << 30)
    # warm up both paths (library load, kernels, allocator, and the weight-term
    # fits of every stream's window sizes: the same seed gives the same streams)
    warm = synth.serving_requests(7, 1000.0, 32)
    cont.serve(warm)
    ser.serve(warm)
    torch.cuda.synchronize()
    sweep = []
    for rate in [float(r) for r in args.rates.split(",")]:
        n = max(200, int(rate * args.seconds))   # at least 200 requests, so p99 is not the maximum
        reqs = synth.serving_requests(7, rate, n)
        cont.templates = serving._Templates(cfg.nbins, "cuda")
        served = cont.serve(reqs)
        rc = serving.latency_stats(served)
        if args.serve_trace:
            with open(args.serve_trace, "a") as fh:
                fh.write(json.dumps({"rate": rate, "trace": serving.request_trace(served)}) + "\n")
        ser.templates = serving._Templates(cfg.nbins, "cuda")
        rs = serving.latency_stats(ser.serve(reqs))
        sweep.append({"rate": rate, "continuous": rc, "serial": rs})
        print(json.dumps({"rate": rate, "continuous_p50_ms": rc["p50_ms"], "continuous_p99_ms": rc["p99_ms"],
                          "serial_p50_ms": rs["p50_ms"], "serial_p99_ms": rs["p99_ms"]}), file=sys.stderr,
              flush=True)
    top = sweep[-1]["continuous"]
    line = {
        "metric": METRIC, "value": top["windows_per_s"], "unit": "windows/s", "n_gpus": 1,
        "steps": len(sweep), "warmup": 1, "ms_per_step": None, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "serve: Poisson tracking requests, 16 streams, frames 640x480..4096x2160, "
                               "target 24..96, 3 scales, search 2-4x, 16 bins, Gaussian K=3 (%s)"
                               % ("separable" if args.gaussian == "separable" else "2-D planes"),
                   "global_batch": None, "seq_len": None, "parallelism": "none"},
        "p50_ms": top["p50_ms"], "p99_ms": top["p99_ms"], "rate": sweep[-1]["rate"],
        "sweep": sweep,
    }
    print(json.dumps(line), flush=True)


def w3_builds(rep_small=10):
    """The build at the multi-scale configuration's size (2048 x 2048 smooth
    noise, 32 bins, one 31 x 31 scale) for Manhattan, exponential and Gaussian:
    carries and planes timed as graphs of back-to-back launches; algorithmic
    bytes = image read + every plane element written once."""
    import torch
    import paper_1705_03524_amd as swih
    from paper_1705_03524_amd.plan import Plan

    def capture(fn):
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            fn()
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            fn()
        torch.cuda.synchronize()
        return g

    W3 = 2048
    w3 = {}
    w3_img = torch.from_numpy(synth_smooth(W3)).cuda()
    for i, kname in enumerate(("manhattan", "exponential", "gaussian")):
        bp = Plan(swih.Config(32, kname, [(WIN, WIN)]), W3, W3)
        # the first timed kernel of a fresh process runs before the clocks have
        # ramped up: ~50 ms of builds beforehand
        for _ in range(150 if i == 0 else 1):
            swih.build(bp.cfg, w3_img, bp.ws, W3, W3, W3)
        torch.cuda.synchronize()
        rep = 2 if kname == "gaussian" else rep_small
        t = {}
        for ph in ("carries", "planes"):
            g = capture(lambda: [swih.build_phase(bp.cfg, w3_img, bp.ws, ph, 0) for _ in range(rep)])
            g.replay()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            for _ in range(3):
                g.replay()
            b.record()
            torch.cuda.synchronize()
            t[ph] = a.elapsed_time(b) / (3 * rep)
            del g
        planes = 4 * bp.nplanes * 32 * (W3 + 1) * (W3 + 1)
        # the Gaussian's emit also writes its FP64 row carries
        if kname == "gaussian":
            planes += gauss_side_bytes(bp.cfg.K, 32, W3, W3)
        build_ms = t["carries"] + t["planes"]
        w3[kname] = {"ms": t, "plane_bytes": planes,
                     "build_gbs": (W3 * W3 + planes) / (build_ms / 1e3) / 1e9,
                     "build_frac": (W3 * W3 + planes) / (build_ms / 1e3) / 1e9 / HBM_PEAK_GBS,
                     "planes_gbs": planes / (t["planes"] / 1e3) / 1e9}
        del bp
        torch.cuda.empty_cache()
    return w3


def bench_builds(args):
    """The 2048 x 2048, 32-bin builds alone (the headline build-bandwidth measurement)."""
    w3 = w3_builds()
    line = {"metric": "IH-build HBM GB/s", "unit": "GB/s", "n_gpus": 1, "higher_is_better": True,
            "data": "synthetic", "dtype": "u32/f32/f64",
            "config": {"workload": "2048x2048 smooth noise, 32 bins, 31x31 scale: Manhattan, exponential, "
                                   "Gaussian K=3 builds (carries + planes)", "parallelism": "none"},
            "value": w3["manhattan"]["build_gbs"], "builds": w3}
    print(json.dumps(line), flush=True)


def bench_sweep(args):
    """The comparison of Sec. 3 on synthetic images: time of the likelihood map
    against window size (Fig. 6: 640x480 and 1024x1024, Manhattan, 16 bins) for
    SWIH (one build serves every window size, then the map), the wedding cake
    (4 rings over the same build's count plane), brute force on the GPU and the
    oracle's brute force on the host (a bounded sample, extrapolated); the
    wedding cake's map error against ring count (Fig. 5) on the 512x512 scene;
    and the paper's one timed shape (a 345x460 region, 61x91 window)."""
    import torch
    import paper_1705_03524_amd as swih
    from paper_1705_03524_amd import synth
    from paper_1705_03524_amd.plan import Plan
    import oracle

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    def cpu_brute_ms(img, w, h, traw, budget_s):
        """Oracle brute force over whole rows of centres for ~budget_s; the full-map
        time extrapolated from its rate."""
        H_, W_ = img.shape
        r, ry = (w - 1) // 2, (h - 1) // 2
        oracle.bc_map(img, NBINS, oracle.MANHATTAN, w, h, traw, rect=(r, ry, r, ry))  # threads up
        t0 = time.perf_counter()
        y, n = ry, 0
        while time.perf_counter() - t0 < budget_s and y <= H_ - 1 - ry:
            oracle.bc_map(img, NBINS, oracle.MANHATTAN, w, h, traw, rect=(r, y, W_ - 1 - r, y))
            n += W_ - 2 * r
            y += 1
        dt = time.perf_counter() - t0
        return dt / n * (W_ - w + 1) * (H_ - h + 1) * 1e3, n

    cfg_all = None
    sizes = ((480, 640), (1024, 1024))
    wins = (11, 21, 31, 41, 61, 81, 101, 151, 201)
    curves = {}
    for (Hs, Ws) in sizes:
        img = synth.rect_scene(5, Hs, Ws)[0]
        d_img = torch.from_numpy(img).cuda()
        cfg_all = swih.Config(NBINS, swih.MANHATTAN, [(w, w) for w in wins])
        plan = Plan(cfg_all, Hs, Ws)
        build_ms = timed(lambda: plan.build(d_img), 5)
        rows = []
        for si, w in enumerate(wins):
            r = (w - 1) // 2
            tc = np.array([[Ws // 2, Hs // 2]], np.int32)
            d_tc = torch.from_numpy(tc).cuda()
            hist, raw = plan.query(si, d_tc)
            traw = raw[0].contiguous()
            rect = plan.valid_rect(si)
            out = torch.empty((Hs - w + 1, Ws - w + 1), dtype=torch.float32, device="cuda")
            map_ms = timed(lambda: plan.match(si, template_raw=traw, rect=rect, out=out), 10)
            ctm = torch.empty((1, NBINS), dtype=torch.float32, device="cuda")
            swih.cake_query(plan.cfg, plan.ws, Hs, Ws, si, 4, d_tc, ctm)
            cout = torch.empty_like(out)
            cake_ms = timed(lambda: swih.cake_match(plan.cfg, plan.ws, Hs, Ws, si, 4, rect, cout, ctm[0]), 10)
            bout = torch.empty_like(out)
            brute_ms = timed(lambda: swih.brute_match(plan.cfg, d_img, si, rect, bout, traw),
                             1 if w >= 101 else 3)
            same = bool(torch.equal(bout, out))
            cpu_ms, cpu_n = cpu_brute_ms(img, w, w, raw[0].cpu().numpy().astype(np.int64),
                                         args.cpu_seconds / len(wins) / len(sizes))
            rows.append({"w": w, "windows": (Hs - w + 1) * (Ws - w + 1), "swih_map_ms": map_ms,
                         "swih_ms": build_ms + map_ms, "cake4_ms": cake_ms, "brute_gpu_ms": brute_ms,
                         "brute_gpu_equals_swih": same, "cpu_oracle_brute_ms_extrapolated": cpu_ms,
                         "cpu_sample_windows": cpu_n})
            print("sweep %dx%d w=%d: swih %.3f ms, cake %.3f ms, brute gpu %.3f ms, cpu %.0f ms" %
                  (Ws, Hs, w, build_ms + map_ms, cake_ms, brute_ms, cpu_ms), file=sys.stderr, flush=True)
        curves["%dx%d" % (Ws, Hs)] = {"swih_build_ms": build_ms, "rows": rows}
        del plan
        torch.cuda.empty_cache()

    # Fig. 5: likelihood-map error of the approximations against the exact map
    img, rects = synth.rect_scene(1, H, W)
    x0, y0, rw, rh, _ = rects[0]
    r = (WIN - 1) // 2
    tc = np.array([[min(max(x0 + rw // 2, r), W - 1 - r), min(max(y0 + rh // 2, r), H - 1 - r)]], np.int32)
    d_img = torch.from_numpy(img).cuda()
    d_tc = torch.from_numpy(tc).cuda()
    plan = Plan(swih.Config(NBINS, swih.MANHATTAN, [(WIN, WIN)]), H, W)
    plan.build(d_img)
    _, raw = plan.query(0, d_tc)
    exact = plan.match(0, template_raw=raw[0].contiguous())
    acc = []
    for n in (1, 2, 3, 4, 6, 8, 12, 16):
        ctm = torch.empty((1, NBINS), dtype=torch.float32, device="cuda")
        swih.cake_query(plan.cfg, plan.ws, H, W, 0, n, d_tc, ctm)
        cm = torch.empty_like(exact)
        swih.cake_match(plan.cfg, plan.ws, H, W, 0, n, plan.valid_rect(0), cm, ctm[0])
        d = (cm - exact).abs()
        acc.append({"rings": n, "max_abs_map_err": float(d.max()), "mean_abs_map_err": float(d.mean())})
    up = Plan(swih.Config(NBINS, swih.UNIFORM, [(WIN, WIN)]), H, W)
    up.build(d_img)
    uh, _ = up.query(0, d_tc)
    um = up.match(0, template=uh[0].contiguous())
    plain = {"max_abs_map_err": float((um - exact).abs().max()), "mean_abs_map_err": float((um - exact).abs().mean())}

    # the paper's timed shape: a 345 x 460 region, 61 x 91 window (Sec. 3)
    PW, PH, pw, ph = 345, 460, 61, 91
    pimg = synth.rect_scene(6, PH, PW)[0]
    d_p = torch.from_numpy(pimg).cuda()
    pp = Plan(swih.Config(NBINS, swih.MANHATTAN, [(pw, ph)]), PH, PW)
    pc = torch.tensor([[PW // 2, PH // 2]], dtype=torch.int32, device="cuda")
    pp.build(d_p)
    _, praw = pp.query(0, pc)
    praw = praw[0].contiguous()
    pout = torch.empty((PH - ph + 1, PW - pw + 1), dtype=torch.float32, device="cuda")
    swih_ms = timed(lambda: (pp.build(d_p), pp.match(0, template_raw=praw, out=pout)), 10)
    bout = torch.empty_like(pout)
    brute_ms = timed(lambda: swih.brute_match(pp.cfg, d_p, 0, pp.valid_rect(0), bout, praw), 3)
    cpu_ms, cpu_n = cpu_brute_ms(pimg, pw, ph, praw.cpu().numpy().astype(np.int64), 2.0)
    line = {
        "metric": "likelihood-map time vs window size (SWIH, wedding cake, brute force)",
        "unit": "ms", "n_gpus": 1, "higher_is_better": False, "dtype": "u32+f64", "data": "synthetic",
        "config": {"workload": "Fig. 6 shape: 640x480 and 1024x1024 scenes, 16 bins, Manhattan, square "
                               "windows 11..201, full map; wedding cake with 4 rings",
                   "parallelism": "none"},
        "curves": curves,
        "cake_accuracy_512_scene_31x31": {"wedding_cake": acc, "plain_histogram": plain},
        "paper_shape_345x460_61x91": {
            "swih_ms": swih_ms, "brute_gpu_ms": brute_ms, "brute_gpu_over_swih": brute_ms / swih_ms,
            "brute_gpu_equals_swih": bool(torch.equal(bout, pout)),
            "cpu_oracle_brute_ms_extrapolated": cpu_ms, "cpu_sample_windows": cpu_n,
            "cpu_cores": int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)),
            "paper_reported_speedup_over_brute_force": 4.5},
    }
    print(json.dumps(line), flush=True)


def bench_track(args):
    """The tracking loop of Sec. 4 on synthetic sequences (640x480, a 31x31 target
    and 3 distractors holding the target's pixel values in reverse spatial order,
    60 frames each, 16 sequences): localisation error and frames per second for
    the plain histogram and the spatially weighted kernels, 3 scales per frame."""
    import torch
    from paper_1705_03524_amd import synth, tracking

    seqs = [synth.track_sequence(100 + s, 60, ndistract=3) for s in range(16)]
    out = {}
    for k in ("uniform", "manhattan", "euclidean", "gaussian_sep", "exponential"):
        errs, succ, frames = [], [], 0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for fr, gt, side in seqs:
            r = tracking.run_sequence(k, fr, gt, side, scales=(0.9, 1.0, 1.1))
            errs.append(r["errors"])
            succ.append(r["success"])
            frames += len(fr) - 1
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        e = np.concatenate(errs)
        out[k] = {"mean_error_px": float(e.mean()), "median_error_px": float(np.median(e)),
                  "success_rate": float(np.mean(succ)), "frames_per_s": frames / dt}
        print("track %s: mean %.2f px, success %.3f, %.0f frames/s" %
              (k, e.mean(), np.mean(succ), frames / dt), file=sys.stderr, flush=True)
    line = {"metric": "tracking localisation error and frames/s (plain vs spatially weighted histograms)",
            "unit": "px", "n_gpus": 1, "higher_is_better": False, "data": "synthetic",
            "config": {"workload": "16 sequences x 60 frames of 640x480, 31x31 target, 3 distractors with the "
                                   "target's values in reverse spatial order, 16 bins, 3 scales, search 1.5 sides",
                       "parallelism": "none"},
            "kernels": out}
    print(json.dumps(line), flush=True)


def run_frame(args, side_kinds=True, builds=True, cpu=True):
    """The 512 x 512 single-frame step (three kernels); returns the JSON line."""
    import torch
    import paper_1705_03524_amd as swih
    from paper_1705_03524_amd.plan import Plan

    img, tc = scene()
    d_img = torch.from_numpy(img).cuda()
    d_tc = torch.tensor([tc], dtype=torch.int32, device="cuda")
    plans = {k: Plan(swih.Config(NBINS, k, [(WIN, WIN)]), H, W) for k in KERNELS}
    maps = {k: torch.empty((H - WIN + 1, W - WIN + 1), dtype=torch.float32, device="cuda")
            for k in KERNELS}
    tmpl = {k: torch.empty(NBINS, dtype=torch.float32, device="cuda") for k in KERNELS}
    traw = {k: torch.empty(NBINS, dtype=torch.uint32, device="cuda") for k in KERNELS}

    def phase(k, name):
        """One launch of a hot-path phase of kernel k (all on the current stream)."""
        p = plans[k]
        if name in ("carries", "planes"):
            swih.build_phase(p.cfg, d_img, p.ws, name, 0)
        elif name == "query":
            if p.integer:
                swih.query(p.cfg, p.ws, H, W, 0, d_tc, None, traw[k].view(1, NBINS))
            else:
                swih.query(p.cfg, p.ws, H, W, 0, d_tc, tmpl[k].view(1, NBINS), None)
        elif p.integer:
            swih.match(p.cfg, p.ws, H, W, 0, p.valid_rect(0), maps[k], template_raw=traw[k])
        else:
            swih.match(p.cfg, p.ws, H, W, 0, p.valid_rect(0), maps[k], template=tmpl[k])

    PHASES = ("carries", "planes", "query", "match")

    # The three kernels' pipelines are independent: with --streams 3 each runs
    # on its own stream (forked from and joined back to the current one), so
    # the short integer pipelines overlap the Gaussian's long kernels and the
    # launch gaps of one pipeline are covered by the others.
    side_streams = [torch.cuda.Stream() for _ in KERNELS[1:]] if args.streams == 3 else []

    def step():
        if not side_streams:
            for k in KERNELS:
                for ph in PHASES:
                    phase(k, ph)
            return
        main = torch.cuda.current_stream()
        for st in side_streams:
            st.wait_stream(main)
        for k, st in zip(KERNELS, [main] + side_streams):
            with torch.cuda.stream(st):
                for ph in PHASES:
                    phase(k, ph)
        for st in side_streams:
            main.wait_stream(st)

    def capture(fn):
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            fn()
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            fn()
        torch.cuda.synchronize()
        return g

    if args.copy_calibration:
        copy_calibration()
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    eager = {k: maps[k].clone() for k in KERNELS}
    # The step (3 kernels x 4 launches) is replayed from one captured HIP graph,
    # so host-side launch cost never starves the device.
    g_step = capture(step)
    for k in KERNELS:
        maps[k].fill_(-1.0)
    g_step.replay()
    torch.cuda.synchronize()
    for k in KERNELS:
        if not torch.equal(maps[k], eager[k]):
            raise RuntimeError("graph replay of the %s step differs from the eager step" % k)
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(args.steps):
        g_step.replay()
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / args.steps
    # Per-kernel launch durations: ROCm graphs carry no timing events, so each
    # phase is captured as its own graph of REP back-to-back launches and timed
    # with events around its replays on the same stream.
    REP = 10
    per = {}
    for k in KERNELS:
        for ph in PHASES:
            g = capture(lambda: [phase(k, ph) for _ in range(REP)])
            g.replay()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            for _ in range(3):
                g.replay()
            b.record()
            torch.cuda.synchronize()
            per[ph + "_" + k] = a.elapsed_time(b) / (3 * REP)
            del g
    for k in KERNELS:
        per["build_" + k] = per["carries_" + k] + per["planes_" + k]

    # Kernels reported beside the step, not part of it: the same Gaussian in
    # separable form (row pass, then a column walk over the row results) and
    # the exponential kernel (four direction-weighted planes per bin).
    def side_kind(kname, timed):
        sp = Plan(swih.Config(NBINS, kname, [(WIN, WIN)]), H, W)
        smap = torch.empty_like(maps["gaussian"])
        stm = torch.empty(NBINS, dtype=torch.float32, device="cuda")

        def side_phase(name):
            if name in ("carries", "planes"):
                swih.build_phase(sp.cfg, d_img, sp.ws, name, 0)
            elif name == "query":
                swih.query(sp.cfg, sp.ws, H, W, 0, d_tc, stm.view(1, NBINS), None)
            else:
                swih.match(sp.cfg, sp.ws, H, W, 0, sp.valid_rect(0), smap, template=stm)

        ms_ = {}
        for ph in PHASES:
            side_phase(ph)
        torch.cuda.synchronize()
        for ph in timed:
            g = capture(lambda: [side_phase(ph) for _ in range(REP)])
            g.replay()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            for _ in range(3):
                g.replay()
            b.record()
            torch.cuda.synchronize()
            ms_[ph] = a.elapsed_time(b) / (3 * REP)
            del g
        return sp, smap, ms_

    extras = {}
    if side_kinds:
        # (the separable form's carries phase launches nothing)
        _, smap, sep_ms = side_kind("gaussian_sep", ("planes", "query", "match"))
        sep_total = sum(sep_ms.values())
        ep, _, exp_ms = side_kind("exponential", PHASES)
        exp_total = sum(exp_ms.values())
        exp_build = exp_ms["carries"] + exp_ms["planes"]
        nwin_ = (H - WIN + 1) * (W - WIN + 1)
        extras["gaussian_separable"] = {
            "ms": sep_ms, "ms_total": sep_total, "windows_per_s": nwin_ / (sep_total / 1e3),
            "speedup_vs_2d_gaussian": (per["build_gaussian"] + per["query_gaussian"] +
                                       per["match_gaussian"]) / sep_total,
            "max_abs_map_diff_vs_2d": float((smap - maps["gaussian"]).abs().max())}
        extras["exponential"] = {
            "ms": exp_ms, "ms_total": exp_total, "windows_per_s": nwin_ / (exp_total / 1e3),
            "ih_build_gbs": (H * W + 4 * ep.nplanes * NBINS * (H + 1) * (W + 1)) / (exp_build / 1e3) / 1e9,
            "planes_gbs": 4 * ep.nplanes * NBINS * (H + 1) * (W + 1) / (exp_ms["planes"] / 1e3) / 1e9}

    w3 = w3_builds(REP) if builds else {}
    if w3:
        extras["ih_build_2048x2048_32bins"] = w3

    nwin = (H - WIN + 1) * (W - WIN + 1)
    value = len(KERNELS) * nwin / (ms / 1e3)
    # Algorithmic bytes of the two Gaussian kernels (5 corner-contracted planes x 16
    # bins, plus the row carries and band-closing rows): the plane build reads the
    # image once and writes every stored element once; the dense map reads every
    # stored element once and writes one float per centre.
    K = plans["gaussian"].cfg.K
    T = GAUSS_PLANES
    plane_bytes = 4 * T * NBINS * (H + 1) * (W + 1)
    kernels = {
        "build": {"kernel": "emit_gauss (Gaussian plane build, %d planes x 16 bins + row carries)" % T,
                  "alg": H * W + plane_bytes + gauss_side_bytes(K, NBINS, H, W), "ms": per["planes_gaussian"],
                  "prefixes": ("emit_gauss",), "unit": "emit_gauss"},
        "match": {"kernel": "k_sweep + match_gauss_fin (Gaussian dense likelihood map, "
                            "482x482 centres; the finalising pass is ~1% of the phase)",
                  "alg": plane_bytes + gauss_side_bytes(K, NBINS, H, W) + 4 * nwin, "ms": per["match_gaussian"],
                  "prefixes": ("k_sweep", "match_gauss_fin"), "unit": "k_sweep"},
    }

    def roof(k):
        achieved = k["alg"] / (k["ms"] / 1e3) / 1e9
        return {"bound": "hbm", "kernel": k["kernel"], "achieved": achieved, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                "traffic": measured_traffic(k["prefixes"], k["unit"]),
                "alg_bytes_per_launch": k["alg"], "avg_launch_ms": k["ms"]}

    dominant = max(kernels, key=lambda n: kernels[n]["ms"])
    other = "build" if dominant == "match" else "match"
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "windows/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32+f32",
        "data": "synthetic",
        "config": {"workload": "512x512 scene, 16 bins, 31x31 windows, Manhattan+Euclidean+Gaussian "
                               "(sigma=w/4, K=3), full Bhattacharyya map of 482x482 centres per kernel",
                   "global_batch": 1, "seq_len": None, "parallelism": "none",
                   "streams": args.streams},
        "roofline": roof(kernels[dominant]),
        "roofline_" + other: roof(kernels[other]),
        "detail_ms": per,
        # IH build (carries + planes) in algorithmic GB/s: image read + planes written
        "ih_build_gbs": {k: (H * W + 4 * plans[k].nplanes * NBINS * (H + 1) * (W + 1)) /
                            (per["build_" + k] / 1e3) / 1e9 for k in KERNELS},
    }
    line.update(extras)
    if cpu:
        line["cpu_baseline"] = cpu_baseline(img, tc, args.cpu_seconds)
    for k in list(plans):
        del plans[k]
    torch.cuda.empty_cache()
    return line


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(got --gpus %d)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    simple = {"batch": bench_batch, "serve": bench_serve, "sweep": bench_sweep, "track": bench_track,
              "builds": bench_builds}
    if args.workload in simple:
        simple[args.workload](args)
        return
    import torch
    import paper_1705_03524_amd as swih

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    swih.load()
    if args.workload == "ceilings":
        print(json.dumps({"metric": "HBM ceilings", "unit": "GB/s", "n_gpus": 1, "ceilings": ceilings()}),
              flush=True)
        return
    if args.workload == "frame":
        line = run_frame(args, side_kinds=not args.no_extras, builds=not args.no_extras,
                         cpu=not args.no_cpu_baseline)
        print(json.dumps(line), flush=True)
        return
    line, img = run_multiscale(args)
    print("multi-scale step: %.3f ms, %.3e windows/s" % (line["ms_per_step"], line["value"]),
          file=sys.stderr, flush=True)
    if not args.no_extras:
        fr = run_frame(args, side_kinds=True, builds=False, cpu=False)
        line["single_frame_512"] = {k: fr[k] for k in fr if k not in ("metric", "n_gpus", "higher_is_better",
                                                                      "scaling", "vs_baseline", "data")}
        print("512x512 step: %.3f ms" % fr["ms_per_step"], file=sys.stderr, flush=True)
        line["ih_build_2048x2048_32bins"] = w3_builds()
        print("2048x2048 builds done", file=sys.stderr, flush=True)
        bt = run_batch(args)
        line["batch"] = {k: bt[k] for k in ("value", "unit", "ms_per_step", "per_frame_windows_per_s",
                                            "speedup_vs_per_frame", "fused_windows_per_s",
                                            "fused_speedup_vs_per_frame", "autotuned_windows_per_s",
                                            "config", "detail")}
        print("batch done", file=sys.stderr, flush=True)
        line["ceilings"] = ceilings()
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline_multiscale(img)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
