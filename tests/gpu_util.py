"""Helpers shared by the GPU parity tests (not collected by pytest)."""
from __future__ import annotations

import sys

import numpy as np
import torch

from paper_2411_19588_amd import rasterizer as R

DEV = "cuda"
IMG_TOL = 1e-4        # absolute, FP32 image vs FP64 oracle (colour and alpha)
DEPTH_RTOL = 1e-4     # depth is compared as |dz| <= 1e-4 * max(1, |z|)


def say(msg: str) -> None:
    print(msg, flush=True)
    sys.stdout.flush()


def to_dev(scene):
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(DEV)
    return dict(means=t(scene.means), scales=t(scene.scales), quats=t(scene.quats), opacity=t(scene.opacity),
                sh=t(scene.sh), medium=t(scene.medium))


def make_rast(scene, cams=None, **cfg):
    return R.Rasterizer(scene.cameras if cams is None else cams, R.RasterConfig(**cfg))


def forward(scene, rast, medium=None):
    d = to_dev(scene)
    med = d["medium"] if medium is None else medium
    rgb, depth, alpha, ctx = rast.forward(d["means"], d["scales"], d["quats"], d["opacity"], d["sh"],
                                          scene.sh_degree, med)
    torch.cuda.synchronize()
    return rgb, depth, alpha, ctx, d


def compare_pixels(gpu_rgb, gpu_depth, gpu_alpha, orc, tol=IMG_TOL, max_ambiguous_frac=1e-3):
    """Element-wise comparison with the oracle's ambiguity variants.

    gpu_* are (P,3), (P,), (P,) numpy arrays for the same pixel list as `orc`.
    A pixel passes if it is within tolerance of the main oracle value or of one
    of the oracle's variants with near-threshold decisions flipped.
    Returns (n_pass_main, n_pass_variant, worst_error) and asserts.
    """
    ref = np.concatenate([orc["rgb"], orc["depth"][:, None], orc["alpha"][:, None]], axis=1)
    got = np.concatenate([gpu_rgb, gpu_depth[:, None], gpu_alpha[:, None]], axis=1).astype(np.float64)
    scale = np.ones_like(ref)
    scale[:, 3] = np.maximum(1.0, np.abs(ref[:, 3]))
    err = np.max(np.abs(got - ref) / scale, axis=1)
    ok = err <= tol
    n_var = 0
    bad = np.nonzero(~ok)[0]
    for k in bad:
        nv = int(orc.get("nvar", np.zeros(len(ref), np.int32))[k])
        for j in range(nv):
            v = orc["var"][k, j]
            s = np.array([1, 1, 1, max(1.0, abs(v[3])), 1])
            if np.max(np.abs(got[k] - v) / s) <= tol:
                ok[k] = True
                n_var += 1
                break
    worst = float(np.max(err[ok & (err <= tol)])) if np.any(ok & (err <= tol)) else 0.0
    n_bad = int(np.count_nonzero(~ok))
    if n_bad:
        k = int(np.nonzero(~ok)[0][0])
        raise AssertionError(f"{n_bad} pixels differ (first {k}: gpu {got[k]} oracle {ref[k]} err {err[k]:.3g})")
    assert n_var <= max(1, max_ambiguous_frac * len(ref)), f"{n_var} ambiguous pixels"
    return int(np.count_nonzero(err <= tol)), n_var, worst


def pixel_list(w, h):
    ys, xs = np.meshgrid(np.arange(h), np.arange(w), indexing="ij")
    return np.stack([xs.ravel(), ys.ravel()], axis=1).astype(np.int32)


def gather_view(rgb, depth, alpha, rast, v, pix):
    """GPU outputs of view v at integer pixels pix (P,2) as numpy (P,3),(P,),(P,)."""
    (r, d, a) = rast.split(rgb, depth, alpha)[v]
    r = r.detach().cpu().numpy()
    d = d.detach().cpu().numpy()
    a = a.detach().cpu().numpy()
    x, y = pix[:, 0], pix[:, 1]
    return r[:, y, x].T.copy(), d[y, x].copy(), a[y, x].copy()


def unambiguous(O, scene, v, G, opts=None, Gz=None):
    """Zero the upstream gradient at pixels whose forward has a near-threshold decision.

    At such pixels FP32 and FP64 may legitimately take different discrete
    decisions (alpha vs 1/255, transmittance vs 1e-4), so their gradients are
    not unique; both sides get the same masked upstream gradient.
    """
    cam = scene.cameras[v]
    orc = O.render(scene, cam, scene.medium[v], opts or O.Options(), variants=1)
    amb = orc["nvar"] > 0
    G = np.array(G, copy=True)
    G[amb] = 0.0
    if Gz is not None:
        Gz = np.array(Gz, copy=True)
        Gz[amb] = 0.0
    return G, Gz, int(amb.sum())


def grad_close(got, ref, rel=1e-3, name=""):
    """Per-element |g - r| <= rel*|r| + rel*rms(r), and block ||g - r|| <= rel*||r||."""
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    rms = float(np.sqrt(np.mean(ref ** 2))) if ref.size else 0.0
    bad = np.abs(got - ref) > rel * np.abs(ref) + rel * rms + 1e-12
    nrm = float(np.linalg.norm(ref))
    blk = float(np.linalg.norm(got - ref)) / max(nrm, 1e-30)
    if np.any(bad) or (nrm > 0 and blk > rel):
        idx = np.unravel_index(np.argmax(np.abs(got - ref)), ref.shape)
        raise AssertionError(f"{name}: {int(bad.sum())}/{ref.size} elements off, block rel {blk:.3g}, "
                             f"worst at {idx}: got {got[idx]} ref {ref[idx]} (rms {rms:.3g})")
    return blk
