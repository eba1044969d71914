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
    update   : fused Adam over all Gaussian and medium parameters whose epilogue
               applies the activations (exp scales, sigmoid opacity) that the
               next step's forward consumes.
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


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", type=int, default=2, help="synthetic workload (2: 1M Gaussians, 1920x1080)")
    ap.add_argument("--tile", type=int, default=16)
    ap.add_argument("--lds-batch", type=int, default=256)
    ap.add_argument("--persistent", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-stride", type=int, default=8, help="oracle sample: every k-th pixel in x and y")
    ap.add_argument("--no-timer", action="store_true", help="skip the per-kernel HIP event timer")
    return ap.parse_args()


def kernel_bytes(name: str, n: int, views: int, K: int, P: int, tiles: int, ncoef: int):
    """Algorithmic HBM bytes one launch of `name` must move (reads + writes).

    n Gaussians, views V, NV = n V entries, K (Gaussian, tile) pairs, P pixels.
    """
    NV = n * views
    param = n * (3 + 3 + 4 + 1 + 3 * ncoef) * 4
    table = {
        # params once + per entry: record 48, count 4, rect 8, depth key 4 (saved) + sort key/value 8
        "project_fwd": param + NV * (48 + 4 + 8 + 4 + 8),
        "depth_sort_hist": NV * 4,
        "depth_sort_scatter": NV * 16,
        "count_scan": NV * (8 + 8) + NV * 8,       # two gathered passes over (order, count), offsets write
        "emit": K * 8 + NV * (4 + 8 + 4 + 8),
        "tile_sort_hist": K * 4,
        "tile_sort_scatter": K * 16,
        "ranges": K * 4 + tiles * 8,
        # outputs + saved state per pixel; the gathered records of traversed pairs are cache-resident
        "composite_fwd": P * (12 + 4 + 4) + P * 28 + tiles * 8,
        "composite_bwd": P * (12 + 28) + NV * 40 + tiles * 36,
        "project_bwd": param + NV * 40 + param,
        "zero_grad2d": NV * 40,
        "medium_reduce": tiles * 36,
    }
    return table.get(name)


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


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU; --gpus {args.gpus} is not supported "
              "(the multi-GPU sharding is described in DESIGN.md, not implemented)", file=sys.stderr)
        print(json.dumps({"error": "only --gpus 1 is supported", "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    from paper_2411_19588_amd import _native as N
    from paper_2411_19588_amd import rasterizer as R
    from paper_2411_19588_amd import optim as OPT
    from paper_2411_19588_amd import synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    log(f"building scene (config {args.config})")
    sc = synth.make_scene(args.config)
    if sc.n_views != 1:
        raise SystemExit("the timed workload is a single-view configuration")
    cam = sc.cameras[0]
    P = cam.width * cam.height
    ncoef = (sc.sh_degree + 1) ** 2
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    target = t(sc.targets[0].reshape(-1))

    groups = [OPT.Group("means", t(sc.means), OPT.LR["means"]),
              OPT.Group("log_scales", t(sc.log_scales), OPT.LR["scales"], "exp"),
              OPT.Group("quats", t(sc.quats), OPT.LR["quats"]),
              OPT.Group("logits", t(sc.logits), OPT.LR["opacity"], "sigmoid"),
              OPT.Group("sh", t(sc.sh), OPT.LR["sh"]),
              OPT.Group("medium", t(sc.medium), OPT.LR["medium"])]
    opt = OPT.FusedAdam(groups)
    G = {g.name: g for g in groups}
    # parameter activation (exp scales, sigmoid opacity) into the activated buffers
    N.check("gs_activate", N.lib().gs_activate(sc.n, ctypes.c_void_p(G["log_scales"].param.data_ptr()),
                                               ctypes.c_void_p(G["logits"].param.data_ptr()),
                                               ctypes.c_void_p(G["log_scales"].activated.data_ptr()),
                                               ctypes.c_void_p(G["logits"].activated.data_ptr()),
                                               ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)))
    cfg = R.RasterConfig(tile=args.tile, lds_batch=args.lds_batch, persistent=args.persistent)
    rast = R.Rasterizer(sc.cameras, cfg, device=dev)
    means, quats, sh, med = G["means"].param, G["quats"].param, G["sh"].param, G["medium"].param
    scales, opac = G["log_scales"].activated, G["logits"].activated
    grad_out = [G["means"].grad, G["log_scales"].grad, G["quats"].grad, G["logits"].grad, G["sh"].grad,
                G["medium"].grad]
    loss = torch.empty(1, dtype=torch.float32, device=dev)
    grad_rgb = torch.empty(3 * P, dtype=torch.float32, device=dev)
    sptr = lambda: ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)

    # capacity: one checked forward sizes the pair list, with headroom for parameter drift
    log("sizing the pair list")
    _, _, _, ctx = rast.forward(means, scales, quats, opac, sh, sc.sh_degree, med)
    _, K0 = rast.read_status(ctx.saved)
    rast.max_pairs = min(N.GS_MAX_PAIRS, int(K0 * 1.2) + 4096)
    del ctx
    log(f"pairs K = {K0} (K/N = {K0 / sc.n:.1f}), capacity {rast.max_pairs}")

    def step():
        rgb, depth, alpha, fctx = rast.forward(means, scales, quats, opac, sh, sc.sh_degree, med, check=False)
        N.check("gs_l1_loss", N.lib().gs_l1_loss(3 * P, ctypes.c_void_p(rgb.data_ptr()),
                                                 ctypes.c_void_p(target.data_ptr()), ctypes.c_void_p(loss.data_ptr()),
                                                 ctypes.c_void_p(grad_rgb.data_ptr()), sptr()))
        rast.backward(fctx, means, scales, quats, opac, sh, med, grad_rgb, out=grad_out)
        opt.step()
        return fctx

    log(f"warmup {args.warmup}")
    for _ in range(args.warmup):
        fctx = step()
    torch.cuda.synchronize()
    timer = None
    if not args.no_timer:
        timer = N.lib().gs_timer_create(40 * (args.steps + 1))
        rast.timer = timer
    log(f"timing {args.steps} steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        fctx = step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    rast.timer = None
    ms = (t1 - t0) * 1e3 / args.steps
    st, K = rast.read_status(fctx.saved)
    if st & N.GS_STATUS_PAIR_OVERFLOW:
        raise SystemExit(f"pair capacity overflowed during the timed steps ({K} > {rast.max_pairs})")
    log(f"{ms:.3f} ms/step, loss {loss.item():.5f}, K {K}")

    kernels = {}
    if timer is not None:
        names = ["project_fwd", "depth_sort_hist", "depth_sort_scan", "depth_sort_scatter", "count_scan", "emit",
                 "tile_sort_hist", "tile_sort_scan", "tile_sort_scatter", "ranges", "composite_fwd", "zero_grad2d",
                 "composite_bwd", "medium_reduce", "project_bwd"]
        for nm in names:
            tot = ctypes.c_double()
            cnt = ctypes.c_int32()
            N.check("gs_timer_read", N.lib().gs_timer_read(timer, nm.encode(), ctypes.byref(tot), ctypes.byref(cnt)))
            if cnt.value:
                kernels[nm] = {"ms_total": tot.value, "launches": cnt.value, "ms_avg": tot.value / cnt.value}
        N.lib().gs_timer_destroy(timer)
    tiles = rast.tile_count()
    roof = None
    if kernels:
        dom = max(kernels, key=lambda k: kernels[k]["ms_total"] / args.steps)
        for nm, kv in kernels.items():
            b = kernel_bytes(nm, sc.n, 1, K, P, tiles, ncoef)
            if b is not None:
                kv["alg_bytes"] = b
                kv["gbs"] = b / (kv["ms_avg"] * 1e-3) / 1e9
        kd = kernels[dom]
        achieved = kd.get("gbs")
        traffic = traffic_for(dom)
        roof = {"kernel": dom, "bound": "hbm", "achieved": round(achieved, 1) if achieved else None,
                "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4) if achieved else None,
                "traffic": traffic, "alg_bytes_per_launch": kd.get("alg_bytes"),
                "avg_launch_ms": round(kd["ms_avg"], 4)}
        log("per-kernel ms/step: " + ", ".join(f"{k} {v['ms_total'] / args.steps:.3f}" for k, v in kernels.items()))

    cpu = None
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a pixel sample")
        cpu = cpu_baseline(sc, sc.targets[0], args.cpu_stride)
        log(f"oracle {cpu['value'] * 1e6:.0f} pix/s on {cpu['cores']} threads")

    rec = {
        "metric": "fwd+bwd Mpix/s at 1M Gaussians 1080p",
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
        "config": {"workload": f"{sc.n} Gaussians SH{sc.sh_degree}, {cam.width}x{cam.height}, 1 view, "
                               "training step (forward + L1 + backward + fused Adam)",
                   "n_gaussians": sc.n, "sh_degree": sc.sh_degree, "width": cam.width, "height": cam.height,
                   "views": 1, "tile": args.tile, "lds_batch": args.lds_batch, "persistent": bool(args.persistent),
                   "pairs": int(K), "pairs_per_gaussian": round(K / sc.n, 2)},
        "roofline": roof,
        "cpu_baseline": cpu,
        "kernels_ms_per_step": {k: round(v["ms_total"] / args.steps, 4) for k, v in kernels.items()},
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
