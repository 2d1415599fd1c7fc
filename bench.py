"""Benchmark: forward + backward of the volumetric Gaussian rasteriser.

Headline workload: one 1920x1080 view of a 1M-Gaussian clustered scene with
SH degree 3 (the single-view configuration of the paper's method at the scale
of its scenes), inputs resident in HBM.  One step = vgr_render_forward +
vgr_render_backward (preprocess, depth sort, binning, tile sort, ranges,
rasteriser forward, rasteriser backward, preprocess backward), the backward
writing the parameter gradients (no separate zeroing).  Also reported: batched multi-view throughput (16
mixed-resolution views of a 3M-Gaussian scene in one call) against the same
16 views rendered by separate single-view calls, and the FP64 oracle timed
on a bounded pixel sample of the headline frame on the host cores.

Prints one JSON line.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Algorithmic FP32 work per (pixel, Gaussian) pair of the rasteriser, counted
# from its operation list (FMA = 2 flops; add, sub, mul, compare, min = 1;
# each rsq / exp2 / rcp = 1):
#   bound pre-test of every visited pair: row offset d_y (2), the form
#     f = d_y (Q11 d_y + f1) + f0 (4), the comparison (1)              7
#   per lane and Gaussian, shared by the lane's pixels: column offset d_x
#     (2), f0 = d_x (Q00 d_x + 2 l0) - 1 (4), f1 = 2 Q01 d_x + 2 l1 (2)  8 / pixels-per-lane
#   closed-form integral of pairs past the pre-test: a = A d, w = v0 + a,
#     n = v0 x a, |n|^2, |w|^2 (37), rsq (1), exponent and exp2 (4),
#     K' |u| r exp2 (3), skip compare (1)                              46
#   forward compositing of blended pairs (clamp, exp2, T(1-a), stop test,
#     alpha, weight, colour FMAs)                                      12   (X-ray sum: 1)
#   backward of blended pairs: compositing replay (clamp, exp2, rcp, T,
#     g.c, dL/dalpha, colour gradient, g.(colour behind) update) 25 (X-ray:
#     1), moment accumulation (t, sum t, z = mz (w x n)/|w|^2, w/|w|, Z, M) 54
#   a backward that reuses the forward's pre-test masks (colour mode, or one
#     pixel per lane) tests nothing and recomputes d_x, d_y (4) per pair past
#     the pre-test                                                      4
F_TEST, F_SHARED, F_FULL, F_OFFSETS = 7, 8, 46, 4
F_BLEND_FWD = {"color": 12, "xray": 1}
F_BLEND_BWD = {"color": 25 + 54, "xray": 1 + 54}
PEAK_FP32 = 157.3e12    # MI355X published FP32 vector peak (FLOP/s)
CALIB_COPY_BYTES = 1 << 28   # plain device copy used to calibrate the HBM byte counters
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_raster_8x8_1M_1080p.json")


def _kernel_source_hash():
    import hashlib
    src = os.path.join(ROOT, "paper_2412_03378_amd", "csrc", "raster.hip")
    return hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]


def _traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary,
    or None if the kernel source changed since the counters were taken."""
    import json as _json
    try:
        t = _json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    if t.get("raster_source_sha256_16") != _kernel_source_hash():
        return None
    k = t.get("kernels", {}).get(kernel)
    return None if k is None else k.get("bytes_per_launch")


def _flops(tested, full, blended, ppl, mode, direction):
    fb = F_BLEND_FWD[mode] if direction == "fwd" else F_BLEND_BWD[mode]
    offs = F_OFFSETS if direction == "bwd" and (mode == "color" or ppl == 1) else 0
    return tested * (F_TEST + F_SHARED / ppl) + full * (F_FULL + offs) + blended * fb


def _raster_rates(r, call, ppl, mode):
    """TFLOP/s of algorithmic work and fraction of PEAK_FP32 for both
    rasterisers over one eager call: stage times from HIP events on the
    library stream, pair counts from the instrumented kernels on the same
    inputs."""
    r.set_timing(True)
    call()
    stages = r.timing()
    r.set_timing(False)
    r.set_counting(True)
    call()
    st = r.stats()
    r.set_counting(False)
    fl = {"raster_fwd": _flops(st["pairs_tested"], st["pairs_full"], st["pairs_blended"], ppl,
                               mode, "fwd"),
          "raster_bwd": _flops(st["bwd_pairs_tested"], st["bwd_pairs_full"],
                               st["bwd_pairs_blended"], ppl, mode, "bwd")}
    out = {}
    for k, f in fl.items():
        if stages.get(k):
            rate = f / (stages[k] * 1e-3)
            out[k] = {"ms": round(stages[k], 4), "tflops": round(rate / 1e12, 2),
                      "frac": round(rate / PEAK_FP32, 4)}
    return out


def _device_scene(sc, dev, torch):
    import numpy as np
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(dev)
    sh = t(sc.sh) if sc.sh is not None else None
    return [t(sc.means), t(sc.quats), t(sc.scales), t(sc.dens), sh]


def _step(r, params, grads, cams, st, dLs):
    r.forward(*params, cams, st)
    r.backward(dLs, *grads, accumulate=False)   # overwrites: no zeroing needed


def _log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def bench_headline(args, torch, dev):
    from paper_2412_03378_amd import Renderer, Settings, scenes
    _log("generating the 1M-Gaussian 1080p scene")
    wl = scenes.config2()
    params = _device_scene(wl.scene, dev, torch)
    dLs = [torch.from_numpy(d).to(dev) for d in wl.dL]
    grads = [torch.zeros_like(p) for p in params]
    tile = tuple(args.tile)
    st = Settings(sh_degree=3, tile=tile, batch=args.batch)
    r = Renderer(0)
    cams = wl.cams
    _log("warm-up")
    for _ in range(args.warmup):
        _step(r, params, grads, cams, st, dLs)
    torch.cuda.synchronize()
    _log("timed steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        _step(r, params, grads, cams, st, dLs)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1e3 / args.steps
    # stage split from HIP events, in separate steps (the events cost time)
    r.set_timing(True)
    for _ in range(args.steps):
        _step(r, params, grads, cams, st, dLs)
    stages = r.timing()
    r.set_timing(False)
    # pair counts of the same inputs, instrumented kernels, outside the timed region
    r.set_counting(True)
    _step(r, params, grads, cams, st, dLs)
    stats = r.stats()
    r.set_counting(False, wg_timing=True)
    _step(r, params, grads, cams, st, dLs)
    lb = r.stats()
    stats["load_balance_fwd"], stats["load_balance_bwd"] = lb["load_balance_fwd"], lb["load_balance_bwd"]
    r.set_counting(False)
    ppl = tile[0] * tile[1] / 64.0
    fl_fwd = _flops(stats["pairs_tested"], stats["pairs_full"], stats["pairs_blended"], ppl,
                    "color", "fwd")
    fl_bwd = _flops(stats["bwd_pairs_tested"], stats["bwd_pairs_full"],
                    stats["bwd_pairs_blended"], ppl, "color", "bwd")
    # the same step captured once in a hipGraph and replayed (no host work)
    outs = [torch.empty((3, c.height, c.width), device=dev) for c in cams]
    r.graph_capture(params, cams, st, outs, dLs, grads, capacity_factor=1.05, zero_grads=True)
    graph_ms = _graph_time(r, args.steps, torch) * 1e3
    kern = {"raster_fwd": fl_fwd, "raster_bwd": fl_bwd}
    dom = max(kern, key=lambda k: stages.get(k, 0.0))
    achieved = kern[dom] / (stages[dom] * 1e-3)
    roofline = {"bound": "alu", "kernel": dom, "achieved": achieved / 1e12, "peak": PEAK_FP32 / 1e12,
                "unit": "TFLOP/s", "frac": achieved / PEAK_FP32, "traffic": _traffic(dom),
                "flops_per_launch": kern[dom], "launch_ms": stages[dom]}
    splat_ab = (None if args.no_splat else
                _splat_ab(r, params, wl, tile, args.steps, torch, dev, grads, dLs))
    near_ab = None
    if not args.no_splat:
        _log("A/B: near-plane segment off vs on")
        near_ab = {"workload": "single view 1920x1080, 1M Gaussians, SH3 (none near the plane: "
                               "the cost of the option's kernels)",
                   "off": _ab_leg(r, params, wl.cams, Settings(sh_degree=3, tile=tile),
                                  args.steps, torch, grads, dLs),
                   "on": _ab_leg(r, params, wl.cams,
                                 Settings(sh_degree=3, tile=tile, near_segment=True),
                                 args.steps, torch, grads, dLs)}
        near_ab["fwd_bwd_ratio"] = round(near_ab["on"]["fwd_bwd_ms"] / near_ab["off"]["fwd_bwd_ms"], 3)
        _log("A/B: per-tile re-sorting off vs on")
        near_ab["tile_resort_on"] = _ab_leg(r, params, wl.cams,
                                            Settings(sh_degree=3, tile=tile, tile_resort=True),
                                            args.steps, torch, grads, dLs)
        near_ab["tile_resort_fwd_bwd_ratio"] = round(
            near_ab["tile_resort_on"]["fwd_bwd_ms"] / near_ab["off"]["fwd_bwd_ms"], 3)
        _log("A/B: per-tile re-sorting with a per-pixel window of 8 (8x8 tiles)")
        near_ab["pixel_window_8"] = _ab_leg(r, params, wl.cams,
                                            Settings(sh_degree=3, tile=(8, 8), tile_resort=True,
                                                     pixel_window=8),
                                            args.steps, torch, grads, dLs)
        near_ab["pixel_window_8_fwd_bwd_ratio"] = round(
            near_ab["pixel_window_8"]["fwd_bwd_ms"] / near_ab["off"]["fwd_bwd_ms"], 3)
    return dict(ms=ms, stages=stages, stats=stats, roofline=roofline, wl=wl, graph_ms=graph_ms,
                flops={"raster_fwd": fl_fwd, "raster_bwd": fl_bwd}, splat_ab=splat_ab,
                near_ab=near_ab)


def _ab_leg(r, params, cams, st, steps, torch, grads, dLs):
    """Forward-only and forward+backward times of one model, with its stage
    split (HIP events, separate steps) and counters."""
    for _ in range(3):
        r.forward(*params, cams, st)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        r.forward(*params, cams, st)
    torch.cuda.synchronize()
    fwd_ms = (time.perf_counter() - t0) * 1e3 / steps
    for _ in range(2):
        _step(r, params, grads, cams, st, dLs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        _step(r, params, grads, cams, st, dLs)
    torch.cuda.synchronize()
    step_ms = (time.perf_counter() - t0) * 1e3 / steps
    r.set_timing(True)
    for _ in range(steps):
        _step(r, params, grads, cams, st, dLs)
    stages = r.timing()
    r.set_timing(False)
    r.set_counting(True)
    r.forward(*params, cams, st)
    stats = r.stats()
    r.set_counting(False)
    pick = ("preprocess_fwd", "sort_tiles", "raster_fwd", "raster_bwd", "preprocess_bwd")
    return {"fwd_ms": round(fwd_ms, 4), "fwd_bwd_ms": round(step_ms, 4),
            "stages_ms": {k: round(stages[k], 4) for k in pick},
            "instances": stats["instances"], "pairs_tested": stats["pairs_tested"],
            "pairs_blended": stats["pairs_blended"]}


def _splat_ab(r, params, wl, tile, steps, torch, dev, grads, dLs):
    """The headline scene with the paper's volumetric opacity and with the
    3DGS splatting opacity it replaces (same pipeline, same GPU).  The
    splats' peak opacity is that of the volumetric model for an isotropic
    Gaussian of the same volume seen through its centre,
    o = 1 - exp(-kappa sqrt(2 pi) (s_x s_y s_z)^(1/3)), so that both scenes are
    about equally opaque."""
    import numpy as np
    from paper_2412_03378_amd import Settings
    _log("A/B: volumetric vs splatting opacity")
    sc = wl.scene
    sg = np.cbrt(np.prod(sc.scales.astype(np.float64), axis=1))
    o = -np.expm1(-sc.dens.astype(np.float64) * math.sqrt(2.0 * math.pi) * sg)
    p_splat = list(params)
    p_splat[3] = torch.from_numpy(o.astype(np.float32)).to(dev)
    vol = _ab_leg(r, params, wl.cams, Settings(sh_degree=3, tile=tile), steps, torch, grads, dLs)
    spl = _ab_leg(r, p_splat, wl.cams, Settings(sh_degree=3, tile=tile, alpha_model="splat"),
                  steps, torch, grads, dLs)
    ratio = lambda k: round(vol["stages_ms"][k] / spl["stages_ms"][k], 3)
    return {"workload": "single view 1920x1080, 1M Gaussians, SH3",
            "volumetric": vol, "splat": spl,
            "fwd_ratio": round(vol["fwd_ms"] / spl["fwd_ms"], 3),
            "fwd_bwd_ratio": round(vol["fwd_bwd_ms"] / spl["fwd_bwd_ms"], 3),
            "raster_fwd_ratio": ratio("raster_fwd"), "raster_bwd_ratio": ratio("raster_bwd")}


def _graph_time(r, steps, torch):
    for _ in range(2):
        r.graph_launch()
    r.graph_check()
    t0 = time.perf_counter()
    for _ in range(steps):
        r.graph_launch()
    r.graph_check()
    return (time.perf_counter() - t0) / steps


def bench_batched(args, torch, dev):
    """16 mixed-resolution views: the tile shape picked by the autotuner, then
    forward + backward of all views captured in one hipGraph and replayed,
    against the same views rendered by separate single-view calls."""
    from paper_2412_03378_amd import Renderer, Settings, scenes
    _log("generating the 3M-Gaussian 16-view scene")
    wl = scenes.config3()
    params = _device_scene(wl.scene, dev, torch)
    dLs = [torch.from_numpy(d).to(dev) for d in wl.dL]
    grads = [torch.zeros_like(p) for p in params]
    outs = [torch.empty((3, c.height, c.width), device=dev) for c in wl.cams]
    r = Renderer(0)
    nv = len(wl.cams)
    _log("autotuning the tile shape")
    tile, batch, tune_ms = r.autotune(params, wl.cams, Settings(sh_degree=3), outs, dLs, grads,
                                      iters=2)
    st = Settings(sh_degree=3, tile=tile, batch=batch)
    res = {"tile": list(tile), "batch": batch, "autotune_ms": [round(x, 3) for x in tune_ms]}
    _log("batched views, one captured graph")
    # load balance over the compute units (workgroup timing, one eager call)
    r.set_counting(False, wg_timing=True)
    r.forward(*params, wl.cams, st)
    r.backward(dLs, *grads, accumulate=False)
    s = r.stats()
    r.set_counting(False)
    res["load_balance"] = {"raster_fwd": round(s["load_balance_fwd"], 3),
                           "raster_bwd": round(s["load_balance_bwd"], 3)}

    def call_all():
        r.forward(*params, wl.cams, st)
        r.backward(dLs, *grads, accumulate=False)
    res["rasterisers"] = _raster_rates(r, call_all, tile[0] * tile[1] / 64.0, "color")
    r.graph_capture(params, wl.cams, st, outs, dLs, grads, capacity_factor=1.1, zero_grads=True)
    res["batched"] = nv / _graph_time(r, args.batched_steps, torch)
    _log("single-view calls")
    # single-view calls get their own launch shape: the 16 calls timed for
    # each shape the autotuner tries, the fastest kept
    def single_calls(stx):
        for k, (c, d) in enumerate(zip(wl.cams, dLs)):
            r.forward(*params, [c], stx)
            r.backward([d], *grads, accumulate=k > 0)
    shapes = [((w, h), bb) for bb in (64, 32) for (w, h) in ((8, 8), (16, 8), (16, 16), (32, 8))]
    single_ms = []
    for (tw, th), bb in shapes:
        stx = Settings(sh_degree=3, tile=(tw, th), batch=bb)
        single_calls(stx)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(2):
            single_calls(stx)
        torch.cuda.synchronize()
        single_ms.append((time.perf_counter() - t0) / 2 * 1e3)
    tile1, batch1 = shapes[min(range(len(shapes)), key=lambda i: single_ms[i])]
    st1 = Settings(sh_degree=3, tile=tile1, batch=batch1)
    res["tile_single"] = list(tile1)
    res["batch_single"] = batch1
    res["single_tune_ms"] = [round(x, 3) for x in single_ms]

    def eager(calls):
        for _ in range(max(1, args.warmup // 2)):
            calls()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.batched_steps):
            calls()
        torch.cuda.synchronize()
        return nv / ((time.perf_counter() - t0) / args.batched_steps)

    def run_single():
        single_calls(st1)
    # like for like: eager against eager (each single-view call waits on the
    # host for its instance count, as the batched call does once), and one
    # captured graph against one captured graph of the 16 single-view calls
    res["single"] = eager(run_single)
    res["batched_eager"] = eager(call_all)
    r.graph_capture_calls(params, wl.cams, [1] * nv, st1, outs, dLs, grads, capacity_factor=1.1,
                          zero_grads=True)
    res["single_graph"] = nv / _graph_time(r, args.batched_steps, torch)
    del params, grads, dLs, outs
    if not args.no_cpu_baseline:
        import oracle
        _log("oracle on one batched view")
        res["oracle"] = oracle_per_view(wl.scene, wl.cams[0], wl.dL[0], 64,
                                        oracle.Settings())
    return res, wl


def bench_xray(args, torch, dev):
    """64 cone-beam projections of a 500k-Gaussian volume, fwd+bwd of all views
    in one call: autotuned tile, stage times from eager calls, throughput from
    a captured hipGraph."""
    from paper_2412_03378_amd import Renderer, Settings, scenes
    _log("generating the 500k-Gaussian X-ray scene")
    wl = scenes.config4()
    params = _device_scene(wl.scene, dev, torch)
    dLs = [torch.from_numpy(d[0]).to(dev) for d in wl.dL]
    grads = [torch.zeros_like(p) for p in params[:4]] + [None]
    outs = [torch.empty((c.height, c.width), device=dev) for c in wl.cams]
    r = Renderer(0)
    _log("autotuning the tile shape (X-ray)")
    xst = Settings(mode="xray", x_min_xray=scenes.XRAY_X_MIN)
    tile, batch, tune_ms = r.autotune(params, wl.cams, xst, outs, dLs, grads, iters=1)
    st = Settings(mode="xray", x_min_xray=scenes.XRAY_X_MIN, tile=tile, batch=batch)
    for _ in range(max(1, args.warmup // 2)):
        _step(r, params, grads, wl.cams, st, dLs)
    torch.cuda.synchronize()
    r.set_timing(True)
    t0 = time.perf_counter()
    for _ in range(args.batched_steps):
        _step(r, params, grads, wl.cams, st, dLs)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.batched_steps
    stages = r.timing()
    r.set_timing(False)
    r.set_counting(True)
    _step(r, params, grads, wl.cams, st, dLs)
    stats = r.stats()
    r.set_counting(False)
    _log("X-ray views, one captured graph")
    r.graph_capture(params, wl.cams, st, outs, dLs, grads, capacity_factor=1.05, zero_grads=True)
    dtg = _graph_time(r, args.batched_steps, torch)
    ppl = tile[0] * tile[1] / 64.0
    fl = {"raster_fwd": _flops(stats["pairs_tested"], stats["pairs_full"], stats["pairs_blended"],
                               ppl, "xray", "fwd"),
          "raster_bwd": _flops(stats["bwd_pairs_tested"], stats["bwd_pairs_full"],
                               stats["bwd_pairs_blended"], ppl, "xray", "bwd")}
    out = {"workload": "X-ray: 64 cone-beam views 512x512, 500k Gaussians, fwd+bwd in one call",
           "x_min": scenes.XRAY_X_MIN,
           "tile": list(tile), "autotune_ms": [round(x, 2) for x in tune_ms],
           "ms_per_step": round(dtg * 1e3, 3), "views_per_s": round(len(wl.cams) / dtg, 1),
           "eager_ms_per_step": round(dt * 1e3, 3),
           "instances": stats["instances"],
           "stages_ms": {k: round(v, 4) for k, v in stages.items()},
           "tflops": {k: round(v / (stages[k] * 1e-3) / 1e12, 2) for k, v in fl.items()
                      if stages.get(k)},
           "frac": {k: round(v / (stages[k] * 1e-3) / PEAK_FP32, 4) for k, v in fl.items()
                    if stages.get(k)}}
    del params, grads, dLs, outs
    if not args.no_cpu_baseline:
        import oracle
        _log("oracle on one X-ray view")
        out["oracle"] = oracle_per_view(wl.scene, wl.cams[0], wl.dL[0], 128,
                                        oracle.Settings(mode="xray",
                                                        x_min_xray=scenes.XRAY_X_MIN))
    return out


def bench_train(args, torch, dev, views_per_call=16):
    """Training-step scale: 6M Gaussians, 64 views 1920x1080, forward + backward
    with the parameter gradients accumulated over all views (4 calls of 16)."""
    from paper_2412_03378_amd import Renderer, Settings, scenes
    _log("generating the 6M-Gaussian 64-view scene")
    wl = scenes.config5()
    params = _device_scene(wl.scene, dev, torch)
    dLs = [torch.from_numpy(d).to(dev) for d in wl.dL]
    grads = [torch.zeros_like(p) for p in params]
    r = Renderer(0)
    nv = len(wl.cams)
    _log("autotuning the tile shape (training calls)")
    outs = [torch.empty((3, c.height, c.width), device=dev) for c in wl.cams[:views_per_call]]
    tile, batch, _ = r.autotune(params, wl.cams[:views_per_call], Settings(sh_degree=3), outs,
                                dLs[:views_per_call], grads, iters=1)
    del outs
    st = Settings(sh_degree=3, tile=tile, batch=batch)

    def step(p, s):
        for v0 in range(0, nv, views_per_call):
            cams = wl.cams[v0:v0 + views_per_call]
            r.forward(*p, cams, s)
            r.backward(dLs[v0:v0 + views_per_call], *grads, accumulate=v0 > 0)

    def timed(p, s):
        step(p, s)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.train_steps):
            step(p, s)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.train_steps
        r.set_timing(True)
        step(p, s)
        stages = r.timing()
        r.set_timing(False)
        return dt, stages

    dt, stages = timed(params, st)
    # the same step as one captured graph of its four 16-view calls
    _log("training step as one captured graph")
    outs = [torch.empty((3, c.height, c.width), device=dev) for c in wl.cams]
    r.graph_capture_calls(params, wl.cams, [views_per_call] * (nv // views_per_call), st, outs,
                          dLs, grads, capacity_factor=1.1, zero_grads=True)
    dt_graph = _graph_time(r, args.train_steps, torch)
    del outs

    def call_one():
        r.forward(*params, wl.cams[:views_per_call], st)
        r.backward(dLs[:views_per_call], *grads, accumulate=True)
    out = {"workload": "training step: 6M Gaussians (1024 clusters), SH3, 64 views 1920x1080, "
                       "fwd+bwd accumulated into FP32 parameter gradients, 16 views per call",
           "tile": list(tile), "batch": batch, "ms_per_step": round(dt * 1e3, 2),
           "views_per_s": round(nv / dt, 1),
           "graph": {"ms_per_step": round(dt_graph * 1e3, 2),
                     "views_per_s": round(nv / dt_graph, 1),
                     "note": "the four 16-view calls captured in one hipGraph and replayed"},
           "rasterisers_one_call": _raster_rates(r, call_one, tile[0] * tile[1] / 64.0, "color")}
    # the same step with the paper's training inputs: theta as the density
    # input (kappa computed in the preprocess) and the densification
    # statistics accumulated by the backward
    # theta is chosen so that kappa is the one of the step above (clamped to
    # theta <= 1 where that kappa is out of reach), so both steps render the
    # same scene and the difference is the cost of the two options
    _log("training step with theta input and densification statistics")
    import numpy as np
    h = (1.0 / wl.scene.scales.astype(np.float64)).mean(1)
    theta = np.clip(-np.expm1(-wl.scene.dens.astype(np.float64) / h) / 0.99, 0.0, 1.0)
    p_theta = list(params)
    p_theta[3] = torch.from_numpy(theta.astype(np.float32)).to(dev)
    gnorm = torch.zeros(wl.scene.n, dtype=torch.float32, device=dev)
    vcount = torch.zeros(wl.scene.n, dtype=torch.int32, device=dev)
    r.set_densify_stats(gnorm, vcount)
    dt2, stages2 = timed(p_theta, Settings(sh_degree=3, tile=tile, batch=batch, density="theta"))
    r.set_densify_stats(None, None)
    pick = lambda d: {k: round(d.get(k, 0.0) * 4, 3) for k in ("preprocess_fwd", "preprocess_bwd")}
    out["stage_ms_per_step"] = {k: round(v * 4, 3) for k, v in stages.items()}
    out["theta_and_densify_stats"] = {
        "ms_per_step": round(dt2 * 1e3, 2), "views_per_s": round(nv / dt2, 1),
        "theta_clamped": int((theta >= 1.0).sum()),
        "stage_ms_per_step": {"kappa": pick(stages), "theta_and_stats": pick(stages2)},
        "note": "theta gives the kappa of the plain step; stage means per call x 4 calls"}
    del params, grads, dLs, p_theta, gnorm, vcount
    if not args.no_cpu_baseline:
        import oracle
        _log("oracle on one training view")
        out["oracle"] = oracle_per_view(wl.scene, wl.cams[0], wl.dL[0], 64, oracle.Settings())
    return out


def _oracle_view_ms(scene, cam, dL, n_pix, st, seed=0):
    """FP64 oracle, forward + backward of one view over all Gaussians,
    extrapolated to the whole view from two random pixel samples (n_pix / 2
    and n_pix pixels, both at least twice the host threads so that the
    per-pixel loop runs on all of them): per pixel (t2 - t1) / (n2 - n1), plus
    the per-view set-up t1 - n1 * per pixel.  dL: (C, H, W).  Returns
    (ms, seconds spent)."""
    import numpy as np
    import oracle
    rng = np.random.default_rng(seed)
    n1 = max(n_pix // 2, 1)

    def run(k):
        pix = np.stack([rng.integers(0, cam.width, k), rng.integers(0, cam.height, k)], 1)
        dLp = np.asarray(dL)[:, pix[:, 1], pix[:, 0]].astype(np.float64)
        t0 = time.perf_counter()
        oracle.render(scene, cam, st, pixels=pix)
        oracle.render_backward(scene, cam, st, dLp, pixels=pix, with_abs=False)
        return time.perf_counter() - t0

    t1 = run(n1)
    t2 = run(n_pix)
    per_pix = max(t2 - t1, 1e-9) / max(n_pix - n1, 1)
    setup = max(t1 - n1 * per_pix, 0.0)
    return (setup + per_pix * cam.width * cam.height) * 1e3, t1 + t2


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(wl, n_pix, n_pix_1core=16):
    """FP64 oracle, forward + backward on n_pix pixels of the headline frame
    (all Gaussians per pixel), extrapolated to the whole frame, on all host
    threads and on one."""
    import oracle
    cam = wl.cams[0]
    total_ms, t_all = _oracle_view_ms(wl.scene, cam, wl.dL[0], n_pix, oracle.Settings())
    threads = oracle.max_threads()
    oracle.set_threads(1)
    try:
        one_ms, t_one = _oracle_view_ms(wl.scene, cam, wl.dL[0], n_pix_1core, oracle.Settings())
    finally:
        oracle.set_threads(threads)
    return {"value": total_ms, "unit": "ms per fwd+bwd (extrapolated)",
            "cores": threads, "kind": "oracle", "cpu_model": _cpu_model(),
            "one_core": {"value": one_ms, "cores": 1,
                         "sample": f"{n_pix_1core // 2} and then {n_pix_1core} pixels "
                                   f"({t_one:.1f} s), extrapolated the same way"},
            "sample": f"fwd+bwd of {n_pix // 2} and then {n_pix} random pixels of the "
                      f"1920x1080 frame over all {wl.scene.n} Gaussians in FP64 ({t_all:.1f} s); "
                      f"per-pixel cost from the difference, scaled to "
                      f"{cam.width * cam.height} pixels plus the per-view set-up"}


def bench_parity(args, torch, dev, calls=200):
    """The parity workload (one 128x128 view, 1000 Gaussians, SH0, 16x16
    tiles, forward only): mean forward time over `calls` eager calls, pair
    counts, and the oracle's whole frame beside it on all host threads and on
    one (no extrapolation)."""
    from paper_2412_03378_amd import Renderer, Settings, scenes
    wl = scenes.config1()
    params = _device_scene(wl.scene, dev, torch)
    r = Renderer(0)
    st = Settings(tile=(16, 16))
    for _ in range(10):
        r.forward(*params, wl.cams, st)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(calls):
        r.forward(*params, wl.cams, st)
    torch.cuda.synchronize()
    us = (time.perf_counter() - t0) / calls * 1e6
    r.set_counting(True)
    r.forward(*params, wl.cams, st)
    stats = r.stats()
    r.set_counting(False)
    out = {"workload": "single view 128x128, 1000 Gaussians, SH0, 16x16 tiles, forward only",
           "forward_us": round(us, 1), "pairs_tested": stats["pairs_tested"],
           "pairs_blended": stats["pairs_blended"]}
    if not args.no_cpu_baseline:
        import oracle
        threads = oracle.max_threads()
        res = {}
        for n in (threads, 1):
            oracle.set_threads(n)
            try:
                t0 = time.perf_counter()
                oracle.render(wl.scene, wl.cams[0], oracle.Settings())
                res[n] = (time.perf_counter() - t0) * 1e3
            finally:
                oracle.set_threads(threads)
        out["oracle"] = {"forward_ms": round(res[threads], 2), "cores": threads,
                         "forward_ms_one_core": round(res[1], 2), "kind": "oracle",
                         "sample": "the whole 128x128 frame over all 1000 Gaussians in FP64"}
    return out


def oracle_per_view(scene, cam, dL, n_pix, st):
    """The oracle beside a multi-view workload: one view, extrapolated, as
    views/s on the host cores."""
    import oracle
    ms, t_all = _oracle_view_ms(scene, cam, dL, n_pix, st)
    return {"views_per_s": round(1e3 / ms, 6), "ms_per_view": round(ms, 1),
            "cores": oracle.max_threads(), "kind": "oracle",
            "sample": f"fwd+bwd of {n_pix // 2} and then {n_pix} random pixels of one "
                      f"{cam.width}x{cam.height} view over all {scene.n} Gaussians in FP64 "
                      f"({t_all:.1f} s), extrapolated as for the headline"}


def write_traffic(fetch_csv, write_csv, out_path=TRAFFIC_FILE):
    """Per-launch HBM bytes of the rasteriser kernels from two rocprofv3 --pmc
    runs of `bench.py --profile` (counter FETCH_SIZE, then WRITE_SIZE; KiB per
    dispatch), each scaled by the reading of the same counter for the plain
    copy of CALIB_COPY_BYTES that the profile run starts with."""
    import csv
    import statistics

    def read(path, counter):
        per = {}
        for row in csv.DictReader(open(path)):
            if row.get("Counter_Name") != counter:
                continue
            name = row.get("Kernel_Name", "")
            per.setdefault(name, []).append(float(row["Counter_Value"]))
        return per

    res = {"raster_source_sha256_16": _kernel_source_hash(), "calibration_bytes": CALIB_COPY_BYTES,
           "kernels": {}}
    for counter, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        per = read(path, counter)
        copies = [v for k, vs in per.items() if "copyBuffer" in k or "copy" in k.lower()
                  for v in vs]
        ref = max(copies) * 1024.0        # KiB -> bytes, the big calibration copy
        scale = CALIB_COPY_BYTES / ref
        res[counter + "_scale"] = scale
        for k, vs in per.items():
            for short in ("raster_fwd_kernel", "raster_bwd_kernel"):
                if short in k and "true>" not in k:       # timed (non-counting) variants
                    key = short.replace("_kernel", "")
                    d = res["kernels"].setdefault(key, {})
                    d[counter + "_KiB_median"] = statistics.median(vs)
                    d[counter.lower() + "_bytes"] = statistics.median(vs) * 1024.0 * scale
    for k, d in res["kernels"].items():
        if "fetch_size_bytes" in d and "write_size_bytes" in d:
            d["bytes_per_launch"] = d["fetch_size_bytes"] + d["write_size_bytes"]
    with open(out_path, "w") as f:
        json.dump(res, f, indent=1)
    print(json.dumps(res))


# Algorithmic HBM bytes per dispatch of the headline step (1M Gaussians, SH3,
# one 1920x1080 view, 8x8 tiles): n = m = 1M items, K instances, 32400 tiles.
#   preprocess: parameters in (means 12, quats 16, scales 12, dens 4, SH 192 B)
#     and record (128 B), depth key, item id, tile count (4 B each) and tile
#     rectangle (8 B) out per Gaussian                      236 + 148 B per item
#   radix scatter: key and value read and written once          16 B per key
#   radix histogram: key read once                               4 B per key
#   emission: key and value written per instance                  8 B per instance
#   ranges: key read per instance                                 4 B per instance
#   record-gradient zeroing: 16 floats per item                 64 B per item
#   preprocess backward: parameters (236 B) and record gradient (64 B) in,
#     parameter gradients (236 B) out                           536 B per item
def algorithmic_bytes(kernel, n_items, n_inst):
    depth = kernel.endswith("<4>")          # the 1M-key depth sort uses 1024-key tiles
    keys = n_items if depth else n_inst
    table = {"preprocess_kernel": 384 * n_items, "radix_scatter_kernel": 16 * keys,
             "radix_hist_kernel": 4 * keys, "emit_kernel": 8 * n_inst, "ranges_kernel": 4 * n_inst,
             "fill_f32_kernel": 64 * n_items, "preprocess_bwd_kernel": 536 * n_items}
    for k, v in table.items():
        if kernel.startswith(k):
            return v
    return None


def _short_kernel(name):
    import re
    k = re.sub(r"^void ", "", name)
    k = re.sub(r"vgr::\(anonymous namespace\)::", "", k)
    return k.split("(")[0].strip()


def profile_summary(root, n_items=1_000_000):
    """Markdown table of every kernel of the `bench.py --profile` run from
    rocprofv3 output under root/{trace,fetch,write,sq}: mean duration (kernel
    trace), HBM bytes per dispatch (FETCH_SIZE and WRITE_SIZE scaled by the
    calibration copy), achieved GB/s and share of 8 TB/s, algorithmic bytes
    where stated, VALU instructions and the FP32 FLOP counter (unit from the
    calibration multiply)."""
    import csv
    import statistics

    def counters(sub):
        per = {}
        for row in csv.DictReader(open(os.path.join(root, sub, "run_counter_collection.csv"))):
            per.setdefault((_short_kernel(row["Kernel_Name"]), row["Counter_Name"]), []).append(
                float(row["Counter_Value"]))
        return per

    stats = {}
    for row in csv.DictReader(open(os.path.join(root, "trace", "run_kernel_stats.csv"))):
        stats[_short_kernel(row["Name"])] = (int(row["Calls"]), float(row["AverageNs"]))
    fetch, write, sq = counters("fetch"), counters("write"), counters("sq")
    copy = "__amd_rocclr_copyBuffer"
    fscale = CALIB_COPY_BYTES / (max(fetch[(copy, "FETCH_SIZE")]) * 1024.0)
    wscale = CALIB_COPY_BYTES / (max(write[(copy, "WRITE_SIZE")]) * 1024.0)
    mul = [k for (k, c) in sq if c == "SQ_INSTS_VALU_FLOPS_FP32" and "MulFunctor" in k]
    flop_unit = None
    if mul:
        v = max(sq[(mul[0], "SQ_INSTS_VALU_FLOPS_FP32")])
        flop_unit = (CALIB_COPY_BYTES // 4) / v if v > 0 else None
    n_inst = None
    lines = []
    rows = []
    for k, (calls, avg_ns) in sorted(stats.items(), key=lambda kv: -kv[1][0] * kv[1][1]):
        if k.startswith("at::native") or k == copy:
            continue
        f = fetch.get((k, "FETCH_SIZE"))
        w = write.get((k, "WRITE_SIZE"))
        fb = statistics.median(f) * 1024.0 * fscale if f else None
        wb = statistics.median(w) * 1024.0 * wscale if w else None
        tot = (fb or 0.0) + (wb or 0.0) if (fb is not None or wb is not None) else None
        valu = sq.get((k, "SQ_INSTS_VALU"))
        flops = sq.get((k, "SQ_INSTS_VALU_FLOPS_FP32"))
        rows.append(dict(kernel=k, calls=calls, us=avg_ns / 1e3, fetch=fb, write=wb, total=tot,
                         valu=statistics.median(valu) if valu else None,
                         flops=statistics.median(flops) if flops else None))
    return rows, fscale, wscale, flop_unit


def print_profile_summary(root, n_inst, n_items=1_000_000):
    rows, fscale, wscale, flop_unit = profile_summary(root, n_items)
    print(f"FETCH_SIZE x {fscale:.4f}, WRITE_SIZE x {wscale:.4f} (256 MiB calibration copy); "
          f"SQ_INSTS_VALU_FLOPS_FP32 x {flop_unit if flop_unit is None else round(flop_unit, 3)} "
          f"= FP32 FLOPs (calibration: one multiply per element of 2^26)\n")
    print("| kernel | calls | mean us | HBM bytes / dispatch | GB/s | of 8 TB/s | algorithmic bytes "
          "| algorithmic GB/s | VALU insts | FP32 FLOPs (counter) |")
    print("|---|---:|---:|---:|---:|---:|---:|---:|---:|---:|")
    for r in rows:
        gbs = r["total"] / (r["us"] * 1e3) if r["total"] is not None else None
        ab = algorithmic_bytes(r["kernel"], n_items, n_inst)
        abs_ = ab / (r["us"] * 1e3) if ab else None
        fl = r["flops"] * flop_unit if (r["flops"] is not None and flop_unit) else None
        fmt = lambda v, f: "-" if v is None else format(v, f)
        print(f"| `{r['kernel']}` | {r['calls']} | {r['us']:.1f} | {fmt(r['total'], '.3g')} | "
              f"{fmt(gbs, '.0f')} | {fmt(None if gbs is None else gbs / 8000.0, '.3f')} | "
              f"{fmt(ab, '.3g')} | {fmt(abs_, '.0f')} | {fmt(r['valu'], '.3g')} | {fmt(fl, '.3g')} |")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--tile", type=int, nargs=2, default=(8, 8))
    ap.add_argument("--batch", type=int, default=64, choices=(32, 64),
                    help="records per rasteriser batch of the headline step")
    ap.add_argument("--batched-steps", type=int, default=3)
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-xray", action="store_true")
    ap.add_argument("--no-train", action="store_true")
    ap.add_argument("--no-splat", action="store_true")
    ap.add_argument("--train-steps", type=int, default=2)
    ap.add_argument("--cpu-pixels", type=int, default=128)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write the counter-based traffic summary from two rocprofv3 --pmc "
                         "counter_collection.csv files and exit")
    ap.add_argument("--profile-summary", nargs=2, metavar=("PROF_DIR", "N_INSTANCES"),
                    help="print the per-kernel table of a profiled run (rocprofv3 output in "
                         "PROF_DIR/{trace,fetch,write,sq}) as markdown and exit")
    ap.add_argument("--profile", action="store_true",
                    help="short run for rocprofv3: one plain device copy of known size "
                         "(counter calibration), then warm-up and timed headline steps only")
    args = ap.parse_args()
    if args.profile_summary:
        print_profile_summary(args.profile_summary[0], int(args.profile_summary[1]))
        return
    if args.traffic_from:
        write_traffic(*args.traffic_from)
        return
    if args.profile:
        args.no_batched = args.no_xray = args.no_train = True
        args.no_cpu_baseline = args.no_splat = True
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(views would shard across GPUs with an all-reduce of parameter "
              "gradients; not built).", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("no HIP device", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda", 0)
    if args.profile:
        src = torch.ones(CALIB_COPY_BYTES // 4, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        # one FP32 multiply per element of a known count: calibrates the unit
        # of the FP32 FLOP counter
        dst.mul_(1.0001)
        torch.cuda.synchronize()
        del src, dst
    h = bench_headline(args, torch, dev)
    out = {
        "metric": "ms per fwd+bwd, 1M Gaussians @1080p; views/sec batched vs single-view",
        "value": round(h["ms"], 4),
        "unit": "ms",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(h["ms"], 4),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "single view 1920x1080, 1M clustered Gaussians (64 clusters), "
                               "SH degree 3, fwd+bwd, upstream N(0,1)",
                   "tile": list(args.tile), "batch": args.batch,
                   "instances": h["stats"]["instances"]},
        "graph_ms_per_step": round(h["graph_ms"], 4),
        "stages_ms": {k: round(v, 4) for k, v in h["stages"].items()},
        "pairs": {k: h["stats"][k] for k in ("pairs_tested", "pairs_full", "pairs_blended",
                                             "visits", "visits_full", "bwd_pairs_tested",
                                             "bwd_pairs_full", "bwd_pairs_blended", "bwd_visits",
                                             "bwd_visits_full")},
        "roofline": h["roofline"],
        # per compute unit: summed workgroup durations of each rasteriser, max / mean
        "load_balance": {"raster_fwd": round(h["stats"]["load_balance_fwd"], 3),
                         "raster_bwd": round(h["stats"]["load_balance_bwd"], 3)},
    }
    if h["splat_ab"] is not None:
        out["splat_ab"] = h["splat_ab"]
    if h["near_ab"] is not None:
        out["near_segment_ab"] = h["near_ab"]
    if not args.no_batched:
        torch.cuda.empty_cache()
        res, wl3 = bench_batched(args, torch, dev)
        out["batched"] = {"workload": "16 views mixed resolution (640x480..1920x1080), 3M "
                                      "Gaussians, SH3, fwd+bwd; batched = one hipGraph "
                                      "replay of all views, single = one call per view",
                          "tile": res["tile"], "batch": res["batch"],
                          "autotune_ms": res["autotune_ms"],
                          "tile_single": res["tile_single"], "batch_single": res["batch_single"],
                          "single_tune_ms": res["single_tune_ms"],
                          "views_per_s_batched": round(res["batched"], 2),
                          "views_per_s_single": round(res["single"], 2),
                          "speedup": round(res["batched"] / res["single"], 3),
                          "like_for_like": {
                              "graph": {"batched": round(res["batched"], 2),
                                        "single": round(res["single_graph"], 2),
                                        "speedup": round(res["batched"] / res["single_graph"], 3),
                                        "note": "one graph of the 16-view call against one "
                                                "graph of the 16 single-view calls"},
                              "eager": {"batched": round(res["batched_eager"], 2),
                                        "single": round(res["single"], 2),
                                        "speedup": round(res["batched_eager"] / res["single"], 3),
                                        "note": "one eager 16-view call against 16 eager "
                                                "single-view calls"}},
                          "load_balance": res["load_balance"],
                          "rasterisers": res["rasterisers"]}
        if "oracle" in res:
            out["batched"]["oracle"] = res["oracle"]
    if not args.no_xray:
        torch.cuda.empty_cache()
        out["xray"] = bench_xray(args, torch, dev)
    if not args.profile:
        out["parity_workload"] = bench_parity(args, torch, dev)
    if not args.no_train:
        torch.cuda.empty_cache()
        out["train"] = bench_train(args, torch, dev)
    if not args.no_cpu_baseline:
        _log("oracle on the host cores")
        out["cpu_baseline"] = cpu_baseline(h["wl"], args.cpu_pixels)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
