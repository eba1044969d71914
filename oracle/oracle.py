"""CPU oracle for the underwater Gaussian rasterizer -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module.  It shares no code with the HIP renderer
(package ``paper_2411_19588_amd``) and never imports it.

Functions (each cites the paper passage it follows):

* :func:`key_path` / :func:`keys` -- (tile, depth) keys of Preliminaries
  "Tiles" (16x16 tiles, Gaussians near a tile are listed for it) and the depth
  order of eq. (3dgs_orig).  The sort is ``numpy`` stable argsort on the 64-bit
  key, with pairs emitted in ascending Gaussian index so equal keys keep index
  order.
* :func:`render` -- brute-force per-pixel evaluation over *all* Gaussians of
  eq. (3dgs_orig), eq. (opacity_impact), eq. (3dgs_uw) and eq. (Depth) in FP64;
  also the clean image J = C_air of eq. (scattering_approx) and, optionally, the
  logistic depth map of the Implementation section as the depth image.
* :func:`backward` -- exact FP64 derivative of :func:`render`; medium terms as
  in the appendix "Partial Derivatives" with the missing factor z restored.
* :func:`fd_grad` -- central differences of :func:`render` (the pin for
  :func:`backward`).
* :func:`activate`, :func:`adam_step`, :func:`l1_loss_grad` -- the parameter
  activations of eq. (opacity_impact) (sigmoid opacity) and exp scales, the
  Adam update named in Sec. Optimization, and the L1 term of
  eq. (3DGSoriginalLoss).

All scene arrays use the synthetic generator's SoA FP32 layout; they are
widened to FP64 here.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gs_oracle.c")
_LIB_PATH = os.path.join(_HERE, "_gs_oracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (no fused multiply-add, IEEE semantics)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fopenmp", "-ffp-contract=off",
                               "-fno-fast-math", "-fPIC", "-shared", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class OrcCam(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("fx", ctypes.c_float), ("fy", ctypes.c_float), ("cx", ctypes.c_float), ("cy", ctypes.c_float),
                ("R", ctypes.c_float * 9), ("t", ctypes.c_float * 3), ("near_z", ctypes.c_float)]


class OrcOpts(ctypes.Structure):
    _fields_ = [("tile_w", ctypes.c_int32), ("tile_h", ctypes.c_int32), ("depth_mode", ctypes.c_int32),
                ("sh_degree", ctypes.c_int32), ("kappa_f32", ctypes.c_float), ("dilation_f32", ctypes.c_float),
                ("alpha_min", ctypes.c_double), ("alpha_max", ctypes.c_double), ("t_min", ctypes.c_double),
                ("dilation", ctypes.c_double), ("band", ctypes.c_double), ("depth_output", ctypes.c_int32)]


class OrcScene(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("means", ctypes.c_void_p), ("scales", ctypes.c_void_p),
                ("quats", ctypes.c_void_p), ("opacity", ctypes.c_void_p), ("sh", ctypes.c_void_p)]


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        i64 = ctypes.c_int64
        L.orc_key_path.argtypes = [i64, P, P, P, ctypes.POINTER(OrcCam), ctypes.POINTER(OrcOpts), P, P, P]
        L.orc_project.argtypes = [ctypes.POINTER(OrcScene), ctypes.POINTER(OrcCam), ctypes.POINTER(OrcOpts),
                                  P, P, P, P, P, P]
        L.orc_render.argtypes = [ctypes.POINTER(OrcScene), ctypes.POINTER(OrcCam), P, ctypes.POINTER(OrcOpts),
                                 i64, P, P, P, P, P, P, P, P, ctypes.c_int32, P, P]
        L.orc_backward_pixels.argtypes = [ctypes.POINTER(OrcScene), ctypes.POINTER(OrcCam), P,
                                          ctypes.POINTER(OrcOpts), i64, P, P, P, P, P, P]
        L.orc_backward_project.argtypes = [ctypes.POINTER(OrcScene), ctypes.POINTER(OrcCam),
                                           ctypes.POINTER(OrcOpts), P, P, P, P, P, P]
        L.orc_sh_basis.argtypes = [ctypes.c_int, i64, P, P]
        L.orc_num_threads.restype = ctypes.c_int
        _lib = L
    return _lib


@dataclasses.dataclass
class Options:
    """Discrete rules of the rasterizer (readings of what the paper leaves to 3DGS)."""
    tile_w: int = 16
    tile_h: int = 16
    alpha_min: float = 1.0 / 255.0
    alpha_max: float = 0.99
    t_min: float = 1e-4
    dilation: float = 0.3
    kappa: float = 11.1
    depth_mode: int = 0
    band: float = 1e-5       # relative margin around a threshold inside which a decision is flagged
    depth_output: int = 0     # 0: depth image = the medium's z; 1: logistic map of zhat (visualisation)

    def c(self, sh_degree: int) -> OrcOpts:
        return OrcOpts(self.tile_w, self.tile_h, self.depth_mode, sh_degree, np.float32(self.kappa),
                       np.float32(self.dilation), self.alpha_min, self.alpha_max, self.t_min,
                       float(np.float32(self.dilation)), self.band, self.depth_output)


def _cam(c) -> OrcCam:
    R = np.asarray(c.R, np.float32).reshape(9)
    t = np.asarray(c.t, np.float32).reshape(3)
    return OrcCam(int(c.width), int(c.height), np.float32(c.fx), np.float32(c.fy), np.float32(c.cx),
                  np.float32(c.cy), (ctypes.c_float * 9)(*R), (ctypes.c_float * 3)(*t), np.float32(c.near))


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


class _SceneAoS:
    """FP64 array-of-structures copy of a scene (kept alive while C reads it)."""

    def __init__(self, means, scales, quats, opacity, sh, sh_degree):
        self.means = np.ascontiguousarray(np.asarray(means, np.float64).T)
        self.scales = np.ascontiguousarray(np.asarray(scales, np.float64).T)
        self.quats = np.ascontiguousarray(np.asarray(quats, np.float64).T)
        self.opacity = np.ascontiguousarray(np.asarray(opacity, np.float64))
        self.sh = np.ascontiguousarray(np.asarray(sh, np.float64).T)
        self.sh_degree = int(sh_degree)
        self.n = self.means.shape[0]
        self.c = OrcScene(self.n, _ptr(self.means), _ptr(self.scales), _ptr(self.quats),
                          _ptr(self.opacity), _ptr(self.sh))

    @classmethod
    def of(cls, scene, **over):
        d = dict(means=scene.means, scales=scene.scales, quats=scene.quats, opacity=scene.opacity,
                 sh=scene.sh, sh_degree=scene.sh_degree)
        d.update(over)
        return cls(**d)


# ---------------------------------------------------------------------------
# Keys (Preliminaries, "Tiles"; depth order of eq. 3dgs_orig)
# ---------------------------------------------------------------------------
def key_path(scene, cam, opts: Options = Options(), **over):
    """FP32 depth bits, tile rectangle [x0,y0,x1,y1] (empty when x0>x1) and cull flag per Gaussian."""
    S = _SceneAoS.of(scene, **over)
    n = S.n
    dbits = np.zeros(n, np.uint32)
    rect = np.zeros((n, 4), np.int32)
    culled = np.zeros(n, np.uint8)
    o = opts.c(S.sh_degree)
    c = _cam(cam)
    lib().orc_key_path(n, _ptr(S.means), _ptr(S.scales), _ptr(S.quats), ctypes.byref(c), ctypes.byref(o),
                       _ptr(dbits), _ptr(rect), _ptr(culled))
    return dbits, rect, culled.astype(bool)


def tiles_of(cam, opts: Options = Options()):
    return (-(-cam.width // opts.tile_w), -(-cam.height // opts.tile_h))


def keys(scene, cams: Optional[Sequence] = None, opts: Options = Options()):
    """All (key, value) pairs over the views, sorted ascending (stable).

    key = (global tile id << 32) | FP32 depth bits, value = v * N + g, where the
    global tile id numbers the tiles of view 0 row-major, then view 1, ...
    Returns (keys u64[K], values u32[K], tile_counts i64[total_tiles]).
    """
    cams = scene.cameras if cams is None else cams
    n = scene.n
    all_k, all_v = [], []
    base = 0
    for vi, cam in enumerate(cams):
        tx, ty = tiles_of(cam, opts)
        dbits, rect, culled = key_path(scene, cam, opts)
        x0, y0, x1, y1 = rect.T.astype(np.int64)
        ok = (~culled) & (x0 <= x1) & (y0 <= y1)
        idx = np.nonzero(ok)[0]
        cnt = ((x1 - x0 + 1) * (y1 - y0 + 1))[idx]
        # emit in ascending Gaussian index, each rectangle row-major
        g_rep = np.repeat(idx, cnt)
        start = np.repeat(np.cumsum(cnt) - cnt, cnt)
        j = np.arange(g_rep.size) - start
        w = np.repeat((x1 - x0 + 1)[idx], cnt)
        tyy = y0[g_rep] + j // w
        txx = x0[g_rep] + j % w
        tile = base + tyy * tx + txx
        all_k.append((tile.astype(np.uint64) << np.uint64(32)) | dbits[g_rep].astype(np.uint64))
        all_v.append((vi * n + g_rep).astype(np.uint32))
        base += tx * ty
    k = np.concatenate(all_k) if all_k else np.zeros(0, np.uint64)
    v = np.concatenate(all_v) if all_v else np.zeros(0, np.uint32)
    order = np.argsort(k, kind="stable")
    k, v = k[order], v[order]
    counts = np.bincount((k >> np.uint64(32)).astype(np.int64), minlength=base)
    return k, v, counts


# ---------------------------------------------------------------------------
# Forward
# ---------------------------------------------------------------------------
def project(scene, cam, opts: Options = Options(), **over):
    S = _SceneAoS.of(scene, **over)
    n = S.n
    out = dict(mean2d=np.zeros((n, 2)), conic=np.zeros((n, 3)), cov=np.zeros((n, 3)),
               color=np.zeros((n, 3)), depth=np.zeros(n), color_clamp=np.zeros((n, 3), np.uint8))
    o = opts.c(S.sh_degree)
    c = _cam(cam)
    lib().orc_project(ctypes.byref(S.c), ctypes.byref(c), ctypes.byref(o), _ptr(out["mean2d"]),
                      _ptr(out["conic"]), _ptr(out["cov"]), _ptr(out["color"]), _ptr(out["depth"]),
                      _ptr(out["color_clamp"]))
    return out


def all_pixels(cam) -> np.ndarray:
    ys, xs = np.meshgrid(np.arange(cam.height), np.arange(cam.width), indexing="ij")
    return np.ascontiguousarray(np.stack([xs.ravel(), ys.ravel()], axis=1).astype(np.int32))


def render(scene, cam, medium, opts: Options = Options(), pixels: Optional[np.ndarray] = None,
           variants: int = 0, **over):
    """Per-pixel brute-force render.  `pixels` is (P, 2) int (u, v); None = full frame.

    Returns a dict of FP64 arrays: rgb (P,3), depth, alpha, cair (P,3), tfinal,
    ncontrib, hash and, if `variants` > 0, nvar (P,) and var (P, variants, 5)
    holding (rgb, depth, alpha) with ambiguous threshold decisions flipped.
    """
    S = _SceneAoS.of(scene, **over)
    pix = all_pixels(cam) if pixels is None else np.ascontiguousarray(np.asarray(pixels, np.int32))
    P = pix.shape[0]
    med = np.ascontiguousarray(np.asarray(medium, np.float64).reshape(9))
    out = dict(rgb=np.zeros((P, 3)), depth=np.zeros(P), alpha=np.zeros(P), cair=np.zeros((P, 3)),
               tfinal=np.zeros(P), ncontrib=np.zeros(P, np.int64), hash=np.zeros(P, np.uint64))
    nv = max(int(variants), 0)
    nvar = np.zeros(P, np.int32)
    var = np.zeros((P, max(nv, 1), 5))
    o = opts.c(S.sh_degree)
    c = _cam(cam)
    lib().orc_render(ctypes.byref(S.c), ctypes.byref(c), _ptr(med), ctypes.byref(o), P, _ptr(pix),
                     _ptr(out["rgb"]), _ptr(out["depth"]), _ptr(out["alpha"]), _ptr(out["cair"]),
                     _ptr(out["tfinal"]), _ptr(out["ncontrib"]), _ptr(out["hash"]), nv, _ptr(nvar), _ptr(var))
    if nv:
        out["nvar"] = nvar
        out["var"] = var
    return out


def image(out, cam):
    """Reshape a full-frame render dict into CHW rgb and HW planes."""
    H, W = cam.height, cam.width
    return (out["rgb"].reshape(H, W, 3).transpose(2, 0, 1), out["depth"].reshape(H, W),
            out["alpha"].reshape(H, W))


# ---------------------------------------------------------------------------
# Backward (appendix "Partial Derivatives", completed)
# ---------------------------------------------------------------------------
def backward(scene, cam, medium, grad_rgb, grad_depth=None, opts: Options = Options(),
             pixels: Optional[np.ndarray] = None, grad_cair=None, **over):
    """Exact FP64 gradients of sum(grad_rgb * rgb) + sum(grad_depth * depth) + sum(grad_cair * cair).

    grad_rgb: (P, 3) for the pixel list (or full frame in row-major order); grad_cair (P, 3)
    is the upstream gradient of the clean image J = C_air of eq. (scattering_approx).
    Returns SoA gradients: means (3,N), scales (3,N), quats (4,N), opacity (N,),
    sh (ncoef*3, N), medium (9,), plus g2d (N, 10) of the 2D quantities.
    """
    S = _SceneAoS.of(scene, **over)
    pix = all_pixels(cam) if pixels is None else np.ascontiguousarray(np.asarray(pixels, np.int32))
    P = pix.shape[0]
    med = np.ascontiguousarray(np.asarray(medium, np.float64).reshape(9))
    grgb = np.ascontiguousarray(np.asarray(grad_rgb, np.float64).reshape(P, 3))
    gdep = None if grad_depth is None else np.ascontiguousarray(np.asarray(grad_depth, np.float64).reshape(P))
    gcair = None if grad_cair is None else np.ascontiguousarray(np.asarray(grad_cair, np.float64).reshape(P, 3))
    n = S.n
    g2d = np.zeros((n, 10))
    gmed = np.zeros(9)
    o = opts.c(S.sh_degree)
    c = _cam(cam)
    L = lib()
    L.orc_backward_pixels(ctypes.byref(S.c), ctypes.byref(c), _ptr(med), ctypes.byref(o), P, _ptr(pix),
                          _ptr(grgb), _ptr(gdep) if gdep is not None else None,
                          _ptr(gcair) if gcair is not None else None, _ptr(g2d), _ptr(gmed))
    ncoef = (S.sh_degree + 1) ** 2
    dm, ds, dq, do, dsh = (np.zeros((n, 3)), np.zeros((n, 3)), np.zeros((n, 4)), np.zeros(n),
                           np.zeros((n, ncoef * 3)))
    L.orc_backward_project(ctypes.byref(S.c), ctypes.byref(c), ctypes.byref(o), _ptr(g2d), _ptr(dm), _ptr(ds),
                           _ptr(dq), _ptr(do), _ptr(dsh))
    return dict(means=dm.T.copy(), scales=ds.T.copy(), quats=dq.T.copy(), opacity=do, sh=dsh.T.copy(),
                medium=gmed, g2d=g2d)


def loss_linear(scene, cam, medium, grad_rgb, grad_depth=None, opts: Options = Options(), pixels=None,
                grad_cair=None, **over):
    """L = <G, C_uw> + <G_z, z> + <G_J, C_air> with the forward above; returns (L, hashes, color clamp flags)."""
    out = render(scene, cam, medium, opts, pixels, **over)
    L = float(np.sum(out["rgb"] * np.asarray(grad_rgb).reshape(-1, 3)))
    if grad_depth is not None:
        L += float(np.sum(out["depth"] * np.asarray(grad_depth).reshape(-1)))
    if grad_cair is not None:
        L += float(np.sum(out["cair"] * np.asarray(grad_cair).reshape(-1, 3)))
    pr = project(scene, cam, opts, **over)
    return L, out["hash"], pr["color_clamp"]


def fd_grad(scene, cam, medium, grad_rgb, field: str, index, grad_depth=None, opts: Options = Options(),
            pixels=None, rel_h: float = 1e-6, grad_cair=None):
    """Central difference of loss_linear w.r.t. one FP64 scalar (field, index).

    `field` is one of means/scales/quats/opacity/sh/medium; `index` a tuple into
    its SoA array.  Returns (value, ok) where ok is False when any discrete
    decision (contributor list, alpha clamp, colour clamp) differs between the
    two evaluations.
    """
    base = dict(means=np.asarray(scene.means, np.float64), scales=np.asarray(scene.scales, np.float64),
                quats=np.asarray(scene.quats, np.float64), opacity=np.asarray(scene.opacity, np.float64),
                sh=np.asarray(scene.sh, np.float64))
    med = np.asarray(medium, np.float64).reshape(9).copy()
    x0 = float(med[index] if field == "medium" else base[field][index])
    h = rel_h * max(1.0, abs(x0))
    vals = []
    sigs = []
    for sgn in (+1.0, -1.0):
        over = {k: v.copy() for k, v in base.items()}
        m2 = med.copy()
        if field == "medium":
            m2[index] = x0 + sgn * h
        else:
            over[field][index] = x0 + sgn * h
        L, hs, cc = loss_linear(scene, cam, m2, grad_rgb, grad_depth, opts, pixels, grad_cair, **over)
        vals.append(L)
        sigs.append((hs.copy(), cc.copy()))
    ok = np.array_equal(sigs[0][0], sigs[1][0]) and np.array_equal(sigs[0][1], sigs[1][1])
    return (vals[0] - vals[1]) / (2.0 * h), ok


def sh_basis(deg: int, dirs: np.ndarray) -> np.ndarray:
    d = np.ascontiguousarray(np.asarray(dirs, np.float64).reshape(-1, 3))
    Y = np.zeros((d.shape[0], 16))
    lib().orc_sh_basis(deg, d.shape[0], _ptr(d), _ptr(Y))
    return Y[:, : (deg + 1) ** 2]


# ---------------------------------------------------------------------------
# Activation, L1 loss, Adam
# ---------------------------------------------------------------------------
def activate(log_scales, logits):
    """scale = exp(log-scale); opacity = sigmoid(logit) (eq. opacity_impact), FP64."""
    ls = np.asarray(log_scales, np.float64)
    lg = np.asarray(logits, np.float64)
    return np.exp(ls), 1.0 / (1.0 + np.exp(-lg))


def l1_loss_grad(pred, target):
    """Mean absolute error of eq. (3DGSoriginalLoss)'s L1 term and its gradient sign(p - t)/numel."""
    p = np.asarray(pred, np.float64)
    t = np.asarray(target, np.float64)
    d = p - t
    return float(np.mean(np.abs(d))), np.sign(d) / d.size


def adam_step(param, grad, m, v, lr, step, beta1=0.9, beta2=0.999, eps=1e-8):
    """Textbook Adam (Kingma & Ba) with bias correction, as named in Sec. Optimization; FP64."""
    p = np.asarray(param, np.float64)
    g = np.asarray(grad, np.float64)
    m1 = beta1 * np.asarray(m, np.float64) + (1.0 - beta1) * g
    v1 = beta2 * np.asarray(v, np.float64) + (1.0 - beta2) * g * g
    mh = m1 / (1.0 - beta1 ** step)
    vh = v1 / (1.0 - beta2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m1, v1


def num_threads() -> int:
    return int(lib().orc_num_threads())
