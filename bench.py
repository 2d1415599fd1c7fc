"""Benchmark: forward + backward of the volumetric Gaussian rasteriser.

Headline workload: one 1920x1080 view of a 1M-Gaussian clustered scene with
SH degree 3 (the single-view configuration of the paper's method at the scale
of its scenes), inputs resident in HBM.  One step = vgr_render_forward +
vgr_render_backward (preprocess, depth sort, binning, tile sort, ranges,
rasteriser forward, rasteriser backward, preprocess backward) plus zeroing
the parameter gradients.  Also reported: batched multi-view throughput (16
mixed-resolution views of a 3M-Gaussian scene in one call) against the same
16 views rendered by separate single-view calls, and the FP64 oracle timed
on a bounded pixel sample of the headline frame on the host cores.

Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Algorithmic FP32 work per (pixel, Gaussian) pair of the rasteriser, counted
# from its operation list (FMA = 2 flops; add, mul, compare, min = 1; each
# rsq / exp2 / rcp = 1):
#   bound test of every visited pair: d_y, a = A d, w = v0 + a, n = v0 x a,
#     |n|^2, |w|^2, the comparison                                   34
#   per lane and Gaussian, shared by the lane's pixels (d_x, A d_x,
#     v0 + A d_x)                                                     7 / pixels-per-lane
#   closed-form integral of pairs past the bound test (rsq, r^2, exponent,
#     exp2, K'|u| r exp2, skip compare)                               9
#   forward compositing of blended pairs (clamp, exp2, T(1-a), stop test,
#     alpha, weight, colour FMAs)                                     12   (X-ray sum: 1)
#   backward of blended pairs: compositing replay (clamp, exp2, rcp, T, dL/dalpha,
#     colour gradient, colour-behind update)                         32   (X-ray: 1)
#     moment accumulation (t, dK', z, w/|w|, Z, M)                   57
F_TEST, F_SHARED, F_FULL = 34, 7, 9
F_BLEND_FWD = {"color": 12, "xray": 1}
F_BLEND_BWD = {"color": 32 + 57, "xray": 1 + 57}
PEAK_FP32 = 157.3e12    # MI355X published FP32 vector peak (FLOP/s)


def _flops(tested, full, blended, ppl, mode, direction):
    fb = F_BLEND_FWD[mode] if direction == "fwd" else F_BLEND_BWD[mode]
    return tested * (F_TEST + F_SHARED / ppl) + full * F_FULL + blended * fb


def _device_scene(sc, dev, torch):
    import numpy as np
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(dev)
    sh = t(sc.sh) if sc.sh is not None else None
    return [t(sc.means), t(sc.quats), t(sc.scales), t(sc.dens), sh]


def _step(r, params, grads, cams, st, dLs):
    for g in grads:
        if g is not None:
            g.zero_()
    r.forward(*params, cams, st)
    r.backward(dLs, *grads)


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
    st = Settings(sh_degree=3, tile=tile)
    r = Renderer(0)
    cams = wl.cams
    _log("warm-up")
    for _ in range(args.warmup):
        _step(r, params, grads, cams, st, dLs)
    torch.cuda.synchronize()
    _log("timed steps")
    r.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        _step(r, params, grads, cams, st, dLs)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    stages = r.timing()
    r.set_timing(False)
    ms = (t1 - t0) * 1e3 / args.steps
    # pair counts of the same inputs, instrumented kernels, outside the timed region
    r.set_counting(True)
    _step(r, params, grads, cams, st, dLs)
    stats = r.stats()
    r.set_counting(False)
    ppl = tile[0] * tile[1] / 64.0
    fl_fwd = _flops(stats["pairs_tested"], stats["pairs_full"], stats["pairs_blended"], ppl,
                    "color", "fwd")
    fl_bwd = _flops(stats["bwd_pairs_tested"], stats["bwd_pairs_full"],
                    stats["bwd_pairs_blended"], ppl, "color", "bwd")
    kern = {"raster_fwd": fl_fwd, "raster_bwd": fl_bwd}
    dom = max(kern, key=lambda k: stages.get(k, 0.0))
    achieved = kern[dom] / (stages[dom] * 1e-3)
    roofline = {"bound": "alu", "kernel": dom, "achieved": achieved / 1e12, "peak": PEAK_FP32 / 1e12,
                "unit": "TFLOP/s", "frac": achieved / PEAK_FP32, "traffic": None,
                "flops_per_launch": kern[dom], "launch_ms": stages[dom]}
    return dict(ms=ms, stages=stages, stats=stats, roofline=roofline, wl=wl,
                flops={"raster_fwd": fl_fwd, "raster_bwd": fl_bwd})


def bench_batched(args, torch, dev):
    from paper_2412_03378_amd import Renderer, Settings, scenes
    _log("generating the 3M-Gaussian 16-view scene")
    wl = scenes.config3()
    params = _device_scene(wl.scene, dev, torch)
    dLs = [torch.from_numpy(d).to(dev) for d in wl.dL]
    grads = [torch.zeros_like(p) for p in params]
    st = Settings(sh_degree=3, tile=tuple(args.tile))
    r = Renderer(0)
    nv = len(wl.cams)
    res = {}
    for mode in ("batched", "single"):
        _log(f"{mode} views")

        def run():
            if mode == "batched":
                _step(r, params, grads, wl.cams, st, dLs)
            else:
                for g in grads:
                    g.zero_()
                for c, d in zip(wl.cams, dLs):
                    r.forward(*params, [c], st)
                    r.backward([d], *grads)
        for _ in range(max(1, args.warmup // 2)):
            run()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.batched_steps):
            run()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.batched_steps
        res[mode] = nv / dt
    del params, grads, dLs
    return res, wl


def cpu_baseline(wl, n_pix):
    """FP64 oracle, forward + backward on n_pix pixels of the headline frame
    (all Gaussians per pixel), extrapolated to the whole frame."""
    import numpy as np
    import oracle
    cam = wl.cams[0]
    rng = np.random.default_rng(0)
    pix = np.stack([rng.integers(0, cam.width, n_pix), rng.integers(0, cam.height, n_pix)], 1)
    dL = wl.dL[0][:, pix[:, 1], pix[:, 0]].astype(np.float64)
    st = oracle.Settings()
    # per-view set-up alone (depth order, precision matrices, colours): one pixel
    t0 = time.perf_counter()
    oracle.render(wl.scene, cam, st, pixels=pix[:1])
    t_setup = time.perf_counter() - t0
    t0 = time.perf_counter()
    oracle.render(wl.scene, cam, st, pixels=pix)
    oracle.render_backward(wl.scene, cam, st, dL, pixels=pix, with_abs=False)
    t_all = time.perf_counter() - t0
    per_pix = max(t_all - 2 * t_setup, 1e-9) / n_pix
    total_ms = (2 * t_setup + per_pix * cam.width * cam.height) * 1e3
    return {"value": total_ms, "unit": "ms per fwd+bwd (extrapolated)",
            "cores": oracle.max_threads(), "kind": "oracle",
            "sample": f"fwd+bwd of {n_pix} random pixels of the 1920x1080 frame over all "
                      f"{wl.scene.n} Gaussians in FP64 ({t_all:.1f} s), scaled to "
                      f"{cam.width * cam.height} pixels plus the per-view set-up"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--tile", type=int, nargs=2, default=(8, 8))
    ap.add_argument("--batched-steps", type=int, default=3)
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--cpu-pixels", type=int, default=128)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(views would shard across GPUs with an all-reduce of parameter "
              "gradients; not built).", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("no HIP device", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda", 0)
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
                   "tile": list(args.tile), "instances": h["stats"]["instances"]},
        "stages_ms": {k: round(v, 4) for k, v in h["stages"].items()},
        "pairs": {k: h["stats"][k] for k in ("pairs_tested", "pairs_full", "pairs_blended",
                                             "bwd_pairs_tested", "bwd_pairs_full",
                                             "bwd_pairs_blended")},
        "roofline": h["roofline"],
    }
    if not args.no_batched:
        torch.cuda.empty_cache()
        res, wl3 = bench_batched(args, torch, dev)
        out["batched"] = {"workload": "16 views mixed resolution (640x480..1920x1080), 3M "
                                      "Gaussians, SH3, fwd+bwd",
                          "views_per_s_batched": round(res["batched"], 2),
                          "views_per_s_single": round(res["single"], 2),
                          "speedup": round(res["batched"] / res["single"], 3)}
    if not args.no_cpu_baseline:
        _log("oracle on the host cores")
        out["cpu_baseline"] = cpu_baseline(h["wl"], args.cpu_pixels)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
