#!/usr/bin/env python3
"""Benchmark of the underwater Gaussian rasterizer on one MI355X.

Workload (default): 1,000,000 Gaussians, SH degree 3, one 1920x1080 view, the
synthetic scene of the "differentiation check" configuration (same
distributions as the 300k-Gaussian training configuration, seeded), per-view
medium coefficients, L1 loss against a seeded random target.

One timed step = a full training step of the hot path, every part in the HIP
library:
    forward  : projection -> depth sort -> pair emission -> tile sort -> ranges
               -> per-tile compositing with the medium and depth epilogue
    loss     : L1 loss value and gradient
    backward : per-tile adjoint -> medium reduction -> projection adjoint
    update   : Adam over every Gaussian and medium parameter group in one
               launch, whose epilogue applies the activations (exp scales,
               sigmoid opacity) that the next step's forward consumes.
Inputs are resident in HBM before the timed region.  `value` = rendered pixels
per second of such steps (Mpix/s).

Also reported: per-kernel times measured with HIP events on the launch stream
over the timed steps, the roofline of the dominant kernel, and the CPU oracle
timed on a bounded pixel sample of the same frame.  Prints ONE JSON line on
stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import ctypes
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# FP32 VALU peak without packed math: 256 CUs x 4 SIMDs x 16 lanes x 2 flops (FMA) x 2.4 GHz.
VALU_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
# Algorithmic FP32 flops of one (pixel, Gaussian) evaluation (FMA = 2): every walked entry
# computes alpha (dx, dy, the quadratic form, exp, opacity, clamp); a blended one also
# updates T and the colour / depth / weight sums (forward) or the adjoint terms (backward).
FLOPS_ALPHA = 12
FLOPS_BLEND_FWD = 12
FLOPS_BLEND_BWD = 49


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", type=int, default=2,
                    help="synthetic workload (2: 1M Gaussians, 1920x1080; 4: 3M Gaussians, 4 views at 1920x1080)")
    ap.add_argument("--tile", type=int, default=16)
    ap.add_argument("--lds-batch", type=int, default=64)
    ap.add_argument("--persistent", action="store_true")
    ap.add_argument("--no-tile-cull", action="store_true", help="bin every tile of each rectangle")
    ap.add_argument("--separate-adam", dest="fused_adam", action="store_false",
                    help="the projection adjoint writes the gradients and the flat Adam kernel updates the "
                         "parameters (default: Adam fused into the adjoint, the SH coefficients stepped from "
                         "the two factors of their gradient)")
    ap.add_argument("--ppl", type=int, default=0, help="pixels per lane in compositing (0 = library default)")
    ap.add_argument("--fetch", choices=["default", "lds", "scalar"], default="default",
                    help="how compositing waves receive the records")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-stride", type=int, default=2, help="oracle sample: every k-th pixel in x and y")
    ap.add_argument("--no-timer", action="store_true", help="skip the per-kernel HIP event timer")
    ap.add_argument("--phases", type=int, default=0,
                    help="depth-progressive binning phases (1 = full binning; 0 = automatic by view count)")
    ap.add_argument("--phase0-shift", type=int, default=0,
                    help="first depth phase = nearest 1/2^shift of the visible Gaussians (0 = library default)")
    ap.add_argument("--eager", action="store_true", help="time eager launches only (no HIP graph replay)")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the 24-view batched-vs-per-view forward+backward comparison")
    ap.add_argument("--batched-steps", type=int, default=5)
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (read MIB, write MIB) three times, to "
                         "calibrate the HBM byte counters of a profiler, and exit")
    return ap.parse_args()


def kernel_bytes(name: str, n: int, views: int, K: int, P: int, tiles: int, ncoef: int, per_step: int = 1,
                 fused: bool = False):
    """Algorithmic HBM bytes one launch of `name` must move (reads + writes), averaged over the
    `per_step` launches a step makes of it.

    n Gaussians, views V, NV = n V entries, K stored (Gaussian, tile) pairs (all phases), P pixels.
    """
    per_step = max(1, per_step)
    NV = n * views
    tile_passes = (int(tiles).bit_length() + 8) // 9   # radix passes (digits of at most 9 bits) over tile ids 0..tiles
    param = n * (3 + 3 + 4 + 1 + 3 * ncoef) * 4
    nsh0 = n * (3 + 3 + 4 + 1) * 4                     # the non-SH parameters
    table = {
        # params once + per entry: record 48, count 4, rect 8, depth key 4 (saved) + sort key/value 8
        "project_fwd": param + NV * (48 + 4 + 8 + 4 + 8),
        "depth_sort_hist": NV * 4,                 # per digit pass: keys read
        "depth_sort_scatter": NV * 16,             # per digit pass: keys and values read and written
        "alive_rows": tiles * 4 + tiles // 4,      # alive flags read, a span per tile row written
        "phase_count": NV * 8,                     # per phase: order + count (or rectangle) per entry
        "count_scan": NV * (4 + 4 + 8),            # per phase: two passes over the counts, offsets write
        "emit": (K * 8) / per_step + NV * 4,
        # every digit pass of every phase's tile sort moves that phase's pairs
        "tile_sort_hist": (K * 4 * tile_passes) / per_step,
        "tile_sort_scatter": (K * 16 * tile_passes) / per_step,
        "commit": (K * 12) / per_step,
        # outputs + saved state per pixel; the gathered records of traversed pairs are cache-resident
        "composite_fwd": (P * (12 + 4 + 4) + P * 29 + tiles * 8) / per_step,
        "composite_bwd": P * (12 + 28) + NV * 40 + tiles * 36,
        # the parameters and the 2D gradients read.  One view without Adam: every gradient
        # written.  With the Adam step fused in: log-scales, quaternions and logits (8 scalars)
        # stepped there (+ 16 B of activated copies), and 10 planes written for adam_sh (one view;
        # the SH coefficients are not read).  Several views: the SH part runs in sh_views; the
        # non-SH parameters read, the 8 gradients (or steps) and 3 + 3 views planes written.
        "project_bwd": (param + NV * 40 + param) if (not fused and views == 1) else (
            (nsh0 + NV * 40 + (n * 8 * 4 * 5 + n * 16 if fused else n * 32) + n * (3 + 3 * views) * 4)
            if views > 1 else (nsh0 + NV * 40 + n * 8 * 4 * 5 + n * 16 + n * 40)),
        # SH coefficients and the means with their moments read and written, 10 planes read
        "adam_sh": n * (3 * ncoef * 24 + 3 * 24 + 40),
        # means and the 3 + 3 views planes read; SH coefficients and means with their moments read
        # and written (fused), or the SH coefficients read and the SH and means gradients written
        "sh_views": n * (12 + (3 + 3 * views) * 4 + (3 * ncoef * 24 + 3 * 24 if fused else 3 * ncoef * 8 + 12)),
        "zero_grad2d": NV * 40,
        "medium_reduce": tiles * 36,
    }
    return table.get(name)


def kernel_flops(name: str, E: int, Cb: int):
    """Algorithmic flops per step of the compositing kernels: E walked evaluations, Cb blended."""
    if name == "composite_fwd":
        return FLOPS_ALPHA * E + FLOPS_BLEND_FWD * Cb
    if name == "composite_bwd":
        return FLOPS_ALPHA * E + FLOPS_BLEND_BWD * Cb
    return None


def source_hash(path: str) -> str:
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def traffic_for(kernel: str):
    """Measured HBM bytes per launch from committed rocprofv3 counter runs, if they match the source."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(p):
        return None
    try:
        t = json.load(open(p))
        ent = t.get(kernel)
        if not ent:
            return None
        src = os.path.join(ROOT, "paper_2411_19588_amd", "csrc", ent["source"])
        if source_hash(src) != ent["source_sha"]:
            return None
        return float(ent["bytes_per_launch"])
    except Exception:
        return None


def cpu_baseline(scene, target, stride: int):
    from oracle import oracle as O
    cam = scene.cameras[0]
    ys, xs = np.meshgrid(np.arange(stride // 2, cam.height, stride), np.arange(stride // 2, cam.width, stride),
                         indexing="ij")
    pix = np.ascontiguousarray(np.stack([xs.ravel(), ys.ravel()], 1).astype(np.int32))
    t0 = time.perf_counter()
    out = O.render(scene, cam, scene.medium[0], pixels=pix)
    tgt = target[:, pix[:, 1], pix[:, 0]].T.astype(np.float64)
    G = np.sign(out["rgb"] - tgt) / (3.0 * cam.width * cam.height)
    O.backward(scene, cam, scene.medium[0], G, pixels=pix)
    dt = time.perf_counter() - t0
    return {"value": len(pix) / dt / 1e6, "unit": "Mpix/s", "cores": O.num_threads(), "kind": "oracle",
            "sample": f"{len(pix)} pixels (every {stride}th pixel in x and y) of the {cam.width}x{cam.height} frame, "
                      f"FP64 brute-force forward + exact backward incl. per-call projection and depth sort; "
                      f"{dt:.1f} s"}


def batched_compare(args, dev):
    """24 views of uneven resolution (1M Gaussians, SH 3): forward + L1 + backward of all views
    in one pipeline (launch shape and depth-phase schedule from the autotuner, one HIP graph)
    against one pipeline per view (24 forward + backward sequences in one HIP graph, same
    configuration).  The per-view side leaves the gradients per view (the batched side sums them over
    the views in its projection adjoint), so it is timed doing less work than the batched one."""
    import torch
    from paper_2411_19588_amd import _native as N
    from paper_2411_19588_amd import autotune as A
    from paper_2411_19588_amd import rasterizer as R
    from paper_2411_19588_amd import synth
    from paper_2411_19588_amd.trainer import RenderStep

    sc = synth.make_scene(3)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    params = dict(means=t(sc.means), scales=t(sc.scales), quats=t(sc.quats), opacity=t(sc.opacity), sh=t(sc.sh))
    med = t(sc.medium)
    tgts = [t(x).reshape(-1) for x in sc.targets]
    tgt_all = torch.cat(tgts)
    sizes = [(c.width, c.height) for c in sc.cameras]
    P = sum(w * h for w, h in sizes)
    log(f"batched: {len(sizes)} views, {P} pixels; autotuning the launch shape")
    measure = A.render_step_timer(params, sc.sh_degree, sc.cameras, med, tgt_all, reps=3, device=dev)
    t0 = time.perf_counter()
    cfg = A.tune_all(measure, R.RasterConfig(), log=log)
    tune_s = time.perf_counter() - t0
    shape = {k: getattr(cfg, k) for k in A.FIELDS}
    log(f"autotuned shape {shape} ({tune_s:.1f} s)")
    stream = torch.cuda.Stream(device=dev)
    K = args.batched_steps

    def time_graph(enqueue_all, warm):
        with torch.cuda.stream(stream):
            sp = ctypes.c_void_p(stream.cuda_stream)
            g = ctypes.c_void_p()
            N.check("gs_graph_begin", N.lib().gs_graph_begin(sp))
            try:
                enqueue_all(stream)
            finally:
                rc = N.lib().gs_graph_end(sp, ctypes.byref(g))
            N.check("gs_graph_end", rc)
            for _ in range(warm):
                N.lib().gs_graph_launch(g, sp)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for _ in range(K):
                N.check("gs_graph_launch", N.lib().gs_graph_launch(g, sp))
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t1) * 1e3 / K
            N.lib().gs_graph_destroy(g)
        return ms

    bs = RenderStep(params, sc.sh_degree, sc.cameras, med, tgt_all, cfg, device=dev)
    with torch.cuda.stream(stream):
        bs.size_capacity(1.25)
    batched_ms = time_graph(lambda s_: bs.enqueue(s_), 2)
    st, _ = bs.status(stream)
    del bs
    log(f"batched: {batched_ms:.3f} ms per forward+backward of {len(sizes)} views")
    per = []
    for v, cam in enumerate(sc.cameras):
        rs = RenderStep(params, sc.sh_degree, [cam], med[v:v + 1], tgts[v], cfg, device=dev)
        with torch.cuda.stream(stream):
            rs.size_capacity(1.25)
        per.append(rs)

    def all_views(s_):
        for rs in per:
            rs.enqueue(s_)

    per_ms = time_graph(all_views, 2)
    st_pv = max(rs.status(stream)[0] for rs in per)
    del per
    torch.cuda.empty_cache()
    log(f"per-view: {per_ms:.3f} ms; speedup {per_ms / batched_ms:.2f}x")
    if st or st_pv:
        raise SystemExit(f"batched comparison reported status {st} / {st_pv}")
    return {"workload": f"{sc.n} Gaussians SH{sc.sh_degree}, {len(sizes)} views of uneven resolution "
                        f"({P} pixels), forward + L1 + backward",
            "views": len(sizes), "pixels": P, "batched_ms": round(batched_ms, 3), "per_view_ms": round(per_ms, 3),
            "speedup": round(per_ms / batched_ms, 3), "batched_mpix_s": round(P / (batched_ms * 1e-3) / 1e6, 1),
            "per_view_mpix_s": round(P / (per_ms * 1e-3) / 1e6, 1), "shape": shape,
            "autotune_s": round(tune_s, 1)}


KERNELS = ["project_fwd", "depth_sort_hist", "depth_sort_scan", "depth_sort_scatter", "alive_rows", "phase_count",
           "count_scan", "emit", "tile_sort_hist", "tile_sort_scan", "tile_sort_scatter", "commit", "composite_fwd",
           "zero_grad2d", "composite_bwd", "medium_reduce", "project_bwd", "adam_sh", "sh_views"]


def read_timer(N, timer):
    out = {}
    for nm in KERNELS:
        tot = ctypes.c_double()
        cnt = ctypes.c_int32()
        N.check("gs_timer_read", N.lib().gs_timer_read(timer, nm.encode(), ctypes.byref(tot), ctypes.byref(cnt)))
        if cnt.value:
            out[nm] = {"ms_total": tot.value, "launches": cnt.value, "ms_avg": tot.value / cnt.value}
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU; --gpus {args.gpus} is not supported "
              "(the path runs on one GPU; sharding over views is not implemented)", file=sys.stderr)
        print(json.dumps({"error": "only --gpus 1 is supported", "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    from paper_2411_19588_amd import _native as N
    from paper_2411_19588_amd import rasterizer as R
    from paper_2411_19588_amd import synth
    from paper_2411_19588_amd.trainer import TrainStep

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.copy_probe:
        n = args.copy_probe * (1 << 20) // 4
        x = torch.rand(n, device=dev)
        y = torch.empty_like(x)
        for _ in range(3):
            torch.mul(x, 1.0, out=y)     # one elementwise kernel: reads n*4 bytes, writes n*4 bytes
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        torch.mul(x, 1.0, out=y)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        print(json.dumps({"copy_probe_bytes_read": n * 4, "copy_probe_bytes_written": n * 4, "launches": 4,
                          "copy_ms": round(ms, 4), "copy_gbs": round(2 * n * 4 / (ms * 1e-3) / 1e9, 1)}))
        return
    log(f"building scene (config {args.config})")
    sc = synth.make_scene(args.config)
    cam = sc.cameras[0]
    P = sum(c.width * c.height for c in sc.cameras)
    sizes = sorted({(c.width, c.height) for c in sc.cameras})
    ncoef = (sc.sh_degree + 1) ** 2
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a))
    cfg = R.RasterConfig(tile=args.tile, lds_batch=args.lds_batch, persistent=args.persistent, phases=args.phases,
                         phase0_shift=args.phase0_shift,
                         pixels_per_lane=args.ppl, record_fetch=args.fetch, tile_cull=not args.no_tile_cull)
    ts = TrainStep(t(sc.means), t(sc.log_scales), t(sc.quats), t(sc.logits), t(sc.sh), t(sc.medium), sc.sh_degree,
                   sc.cameras, torch.cat([t(x).reshape(-1) for x in sc.targets]), cfg, device=dev,
                   fused=args.fused_adam)
    log("sizing the pair list")
    need = ts.size_capacity(1.25)
    log(f"stored pairs {need}, capacity {ts.max_pairs}")
    stream = torch.cuda.Stream(device=dev)          # default priority
    torch.cuda.synchronize()

    # ---- eager steps, with HIP events around every kernel
    with torch.cuda.stream(stream):
        log(f"eager warmup {args.warmup}")
        for _ in range(args.warmup):
            ts.enqueue(stream)
        torch.cuda.synchronize()
        timer = None
        if not args.no_timer:
            timer = N.lib().gs_timer_create(80 * (args.steps + 1))
            ts.timer = timer
        t0 = time.perf_counter()
        for _ in range(args.steps):
            ts.enqueue(stream)
        torch.cuda.synchronize()
        eager_ms = (time.perf_counter() - t0) * 1e3 / args.steps
        ts.timer = None
        kernels = read_timer(N, timer) if timer is not None else {}
        if timer is not None:
            N.lib().gs_timer_destroy(timer)
        log(f"eager: {eager_ms:.3f} ms/step")

        # ---- the same step captured once into a HIP graph and replayed
        ms = eager_ms
        if not args.eager:
            ts.capture(stream)
            for _ in range(args.warmup):
                ts.replay(stream)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                ts.replay(stream)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3 / args.steps
            log(f"graph: {ms:.3f} ms/step")
    st, K = ts.status(stream)
    if st & N.GS_STATUS_PAIR_OVERFLOW:
        raise SystemExit(f"pair capacity overflowed during the timed steps ({K} > {ts.max_pairs})")
    stats = (ctypes.c_int64 * 5)()
    N.check("gs_forward_stats", N.lib().gs_forward_stats(ctypes.byref(ts.opts), ts.n, ts.rast.n_views,
                                                         ts.rast.host_cams,
                                                         ctypes.c_void_p(ts.saved.data_ptr()), ts.saved.numel(),
                                                         stats, ctypes.c_void_p(stream.cuda_stream)))
    # pairs per depth phase (from the stored per-phase tile ranges)
    _, _, rng = ts.rast.export_keys(R.ForwardContext(ts.saved, ts.max_pairs, ts.n, sc.sh_degree), stream)
    rng = rng.to(torch.int64)
    phases, shift = ts.rast.schedule(ts.n)
    phase_pairs = [int((rng[p, :, 1] - rng[p, :, 0]).sum().item()) for p in range(phases)]
    log(f"live pairs per phase: {phase_pairs}")
    # full (single-phase) binning pair count of the same scene, for K/N
    # (the method's rectangle binning, no culling)
    full = R.Rasterizer(sc.cameras, R.RasterConfig(phases=1, tile_cull=False, max_pairs=int(K * 8)), device=dev)
    g = ts.G
    _, _, _, fctx = full.forward(g["means"].param, g["log_scales"].activated, g["quats"].param,
                                 g["logits"].activated, g["sh"].param, sc.sh_degree, g["medium"].param)
    _, K_full = full.read_status(fctx.saved)
    del fctx, full
    log(f"loss {ts.loss.item():.5f}; stored pairs {K}, full-binning pairs {K_full} (K/N {K_full / sc.n:.1f}), "
        f"E/pixel {stats[1] / P:.1f}, blended/pixel {stats[4] / P:.1f}, live pairs {stats[0]}")

    tiles = ts.rast.tile_count()
    E, Cb, K_live = int(stats[1]), int(stats[4]), int(stats[0])
    roof = None
    if kernels:
        dom = max(kernels, key=lambda k: kernels[k]["ms_total"])
        for nm, kv in kernels.items():
            per_step = kv["launches"] // args.steps
            f = kernel_flops(nm, E, Cb)
            if f is not None:
                kv["alg_flops"] = f / max(1, per_step)
                kv["tflops"] = f / (kv["ms_total"] / args.steps * 1e-3) / 1e12
                continue
            b = kernel_bytes(nm, sc.n, sc.n_views, K_live, P, tiles, ncoef, per_step, args.fused_adam)
            if b is not None:
                kv["alg_bytes"] = b
                kv["gbs"] = b / (kv["ms_avg"] * 1e-3) / 1e9
        kd = kernels[dom]
        if "tflops" in kd:
            roof = {"kernel": dom, "bound": "alu", "achieved": round(kd["tflops"], 2), "peak": VALU_PEAK_TFLOPS,
                    "unit": "TFLOP/s", "frac": round(kd["tflops"] / VALU_PEAK_TFLOPS, 4),
                    "traffic": traffic_for(dom), "alg_flops_per_launch": kd["alg_flops"],
                    "avg_launch_ms": round(kd["ms_avg"], 4)}
        else:
            achieved = kd.get("gbs")
            roof = {"kernel": dom, "bound": "hbm", "achieved": round(achieved, 1) if achieved else None,
                    "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4) if achieved else None,
                    "traffic": traffic_for(dom), "alg_bytes_per_launch": kd.get("alg_bytes"),
                    "avg_launch_ms": round(kd["ms_avg"], 4)}
        log("per-kernel ms/step: " + ", ".join(f"{k} {v['ms_total'] / args.steps:.3f}" for k, v in kernels.items()))
        log("compositing TFLOP/s: " + ", ".join(f"{k} {v['tflops']:.2f}" for k, v in kernels.items() if "tflops" in v))

    cpu = None
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a pixel sample")
        cpu = cpu_baseline(sc, sc.targets[0], args.cpu_stride)
        log(f"oracle {cpu['value'] * 1e6:.0f} pix/s on {cpu['cores']} threads")

    batched = None
    if not args.no_batched:
        del ts
        torch.cuda.empty_cache()
        batched = batched_compare(args, dev)

    rec = {
        "metric": "fwd+bwd Mpix/s at 1M Gaussians 1080p; batched-views vs per-view speedup",
        "value": round(P / (ms * 1e-3) / 1e6, 3),
        "unit": "Mpix/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{sc.n} Gaussians SH{sc.sh_degree}, "
                               f"{' + '.join(f'{w}x{h}' for w, h in sizes)}, {sc.n_views} view(s), "
                               "training step (forward + L1 + backward + Adam)",
                   "n_gaussians": sc.n, "sh_degree": sc.sh_degree, "width": cam.width, "height": cam.height,
                   "views": sc.n_views, "tile": args.tile, "lds_batch": args.lds_batch, "persistent": bool(args.persistent),
                   "pixels_per_lane": args.ppl, "record_fetch": args.fetch,
                   "phases": phases, "phase0_shift": shift, "mode": "eager" if args.eager else "hip_graph",
                   "pairs_stored": int(K), "pairs_full_binning": int(K_full),
                   "pairs_per_gaussian": round(K_full / sc.n, 2), "pairs_live": int(stats[0]),
                   "pairs_live_per_phase": phase_pairs,
                   "evals_per_pixel": round(stats[1] / P, 1), "blends_per_pixel": round(stats[4] / P, 1),
                   "tile_cull": bool(cfg.tile_cull), "adam": "fused" if args.fused_adam else "separate"},
        "eager_ms_per_step": round(eager_ms, 4),
        "roofline": roof,
        "cpu_baseline": cpu,
        "batched": batched,
        "kernels_ms_per_step": {k: round(v["ms_total"] / args.steps, 4) for k, v in kernels.items()},
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
