"""Backscatter estimation (Sec. Optimization, appendix "Backscatter Estimation", Alg. 1 and
Alg. 2) and the L_best term of eq. (OurFinalLoss) -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may
import this module.  It shares no code with the HIP library.

What it computes for one view, from the observed image I (3, H, W) and the rendered depth z
(H, W) of eq. (Depth) (0 where no Gaussian contributes):

1. Alg. 1, steps 1-4: I and z resized to `resize_height` rows (0 = full resolution),
   negative values set to 0.
2. Alg. 2: the depth range of the pixels with a depth is cut into edges_num = 10 evenly spaced
   edges (9 clusters); in each cluster the darkest p_dark = 1 % of the pixels (by the norm of
   their RGB triplet) are kept: their depths darkZ and colours Bc.
3. Alg. 1, steps 6-8: the range of darkZ is cut into intervals_num = 25 evenly spaced edges
   (24 intervals); per colour channel and interval, the smallest Bc value and its depth.
4. Alg. 1, steps 9-10: per channel, the nonlinear least-squares fit of
   B_hat = Binf (1 - exp(-Bb z)) to those (z, value) pairs with Binf in [0, 1] and Bb in [0, 5]
   (scipy's bounded trust-region least squares, the library routine, from several starts).

Readings where the paper is silent (each is also listed in the design notes):
* resize: bilinear, half-pixel centres, edges clamped, width round(W * rows / H);
* only pixels with a depth (z > 0 after the resize) take part (a pixel no Gaussian reaches has
  no depth);
* "darkest": the ceil(p_dark * n) pixels of a cluster of n (p_dark rounded to FP32, the product
  in FP64) with the smallest squared norm r^2 + g^2 + b^2 (the norm's order), ties by pixel index;
* intervals: [e_i, e_{i+1}) with the last one closed; the minimum's ties by pixel index;
* every quantity that decides a pixel's cluster, rank or interval is computed in FP32 with the
  fixed operation sequence below (both implementations take those decisions in the same
  precision); the fit is FP64.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.optimize import least_squares

P_DARK = 0.01
EDGES = 10
INTERVALS = 25
RESIZE_HEIGHT = 300
LAMBDA_EST = 0.1

f32 = np.float32


def resized_size(width: int, height: int, rows: int):
    """Output (width, height) of the resize (unchanged for rows = 0 or rows = height)."""
    if rows <= 0 or rows == height:
        return width, height
    return max(1, int(math.floor(width * rows / height + 0.5))), rows


def _axis(n_in: int, n_out: int):
    """Bilinear source indices and weights along one axis, FP32: s = (i + 1/2) (n_in / n_out) - 1/2,
    clamped at 0; i0 = floor(s), i1 = min(i0 + 1, n_in - 1), w = s - i0."""
    r = f32(n_in) / f32(n_out)
    i = np.arange(n_out, dtype=np.float32)
    s = (i + f32(0.5)) * r - f32(0.5)
    s = np.maximum(s, f32(0.0))
    i0 = np.floor(s).astype(np.int64)
    i1 = np.minimum(i0 + 1, n_in - 1)
    w = (s - i0.astype(np.float32)).astype(np.float32)
    return i0, i1, w


def resize(a: np.ndarray, width: int, height: int) -> np.ndarray:
    """Bilinear resize of (..., H, W) FP32 planes to (..., height, width), then max(0, .)."""
    a = np.asarray(a, np.float32)
    H, W = a.shape[-2:]
    if (W, H) == (width, height):
        return np.maximum(a, f32(0.0))
    y0, y1, wy = _axis(H, height)
    x0, x1, wx = _axis(W, width)
    wx_ = wx[None, :]
    wy_ = wy[:, None]
    one = f32(1.0)
    top = (one - wx_) * a[..., y0[:, None], x0[None, :]] + wx_ * a[..., y0[:, None], x1[None, :]]
    bot = (one - wx_) * a[..., y1[:, None], x0[None, :]] + wx_ * a[..., y1[:, None], x1[None, :]]
    out = (one - wy_) * top + wy_ * bot
    return np.maximum(out.astype(np.float32), f32(0.0))


def _bins(z: np.ndarray, lo, hi, n_bins: int) -> np.ndarray:
    """Evenly spaced bins of [lo, hi] in FP32: j = min(n - 1, floor((z - lo) / ((hi - lo) / n)))."""
    step = (f32(hi) - f32(lo)) / f32(n_bins)
    if not step > 0:
        return np.zeros(z.shape, np.int64)
    t = (z.astype(np.float32) - f32(lo)) / step
    return np.minimum(n_bins - 1, np.floor(t).astype(np.int64))


def dark_pixels(I: np.ndarray, z: np.ndarray, p_dark: float = P_DARK, edges: int = EDGES):
    """Alg. 2: flat indices (into the H W pixels) of the darkest pixels of every depth cluster."""
    I = np.asarray(I, np.float32)
    z = np.asarray(z, np.float32).reshape(-1)
    valid = np.nonzero(z > 0)[0]
    if valid.size == 0:
        return valid
    zv = z[valid]
    cl = _bins(zv, zv.min(), zv.max(), edges - 1)
    r, g, b = (I[c].reshape(-1)[valid] for c in range(3))
    q = (r * r + g * g) + b * b                       # FP32, separately rounded
    keep = []
    for c in range(edges - 1):
        members = np.nonzero(cl == c)[0]
        if members.size == 0:
            continue
        n_sel = int(math.ceil(float(f32(p_dark)) * members.size))   # p_dark as FP32, product in FP64
        order = np.lexsort((valid[members], q[members]))   # by (q, pixel index)
        keep.append(valid[members[order[:n_sel]]])
    return np.sort(np.concatenate(keep))


def interval_minima(I: np.ndarray, z: np.ndarray, sel: np.ndarray, intervals: int = INTERVALS):
    """Alg. 1, steps 6-8: per channel, [(depth, value)] of the smallest selected value per interval."""
    z = np.asarray(z, np.float32).reshape(-1)
    dz = z[sel]
    j = _bins(dz, dz.min(), dz.max(), intervals - 1)
    out = []
    for c in range(3):
        v = np.asarray(I[c], np.float32).reshape(-1)[sel]
        pts = []
        for k in range(intervals - 1):
            m = np.nonzero(j == k)[0]
            if m.size == 0:
                continue
            best = m[np.lexsort((sel[m], v[m]))[0]]
            pts.append((float(dz[best]), float(v[best])))
        out.append(pts)
    return out


def model(binf, bb, z):
    return binf * (1.0 - np.exp(-bb * np.asarray(z, np.float64)))


def residual(binf, bb, pts) -> float:
    z = np.array([p[0] for p in pts], np.float64)
    v = np.array([p[1] for p in pts], np.float64)
    return float(np.sum((model(binf, bb, z) - v) ** 2))


def fit(pts):
    """Bounded nonlinear least squares of Binf (1 - exp(-Bb z)) to the points (Binf in [0, 1],
    Bb in [0, 5]); the best of several starts."""
    if not pts:
        return 0.0, 0.0
    z = np.array([p[0] for p in pts], np.float64)
    v = np.array([p[1] for p in pts], np.float64)
    fun = lambda x: x[0] * (1.0 - np.exp(-x[1] * z)) - v
    best = None
    for b0 in (0.05, 0.5, 0.95):
        for s0 in (0.05, 0.5, 2.0, 4.5):
            r = least_squares(fun, [b0, s0], bounds=([0.0, 0.0], [1.0, 5.0]), method="trf", xtol=1e-15,
                              ftol=1e-15, gtol=1e-15, max_nfev=2000)
            if best is None or r.cost < best.cost:
                best = r
    return float(best.x[0]), float(best.x[1])


def estimate(I: np.ndarray, z: np.ndarray, p_dark: float = P_DARK, resize_height: int = RESIZE_HEIGHT,
             edges: int = EDGES, intervals: int = INTERVALS):
    """Alg. 1 for one view: returns (Binf[3], Bb[3], points per channel)."""
    I = np.asarray(I, np.float32)
    z = np.asarray(z, np.float32)
    H, W = z.shape
    w, h = resized_size(W, H, resize_height)
    Ir = resize(I, w, h)
    zr = resize(z, w, h)
    sel = dark_pixels(Ir, zr, p_dark, edges)
    if sel.size == 0:
        return np.zeros(3), np.zeros(3), [[], [], []]
    pts = interval_minima(Ir, zr, sel, intervals)
    binf, bb = np.zeros(3), np.zeros(3)
    for c in range(3):
        binf[c], bb[c] = fit(pts[c])
    return binf, bb, pts


def prior(medium: np.ndarray, est: np.ndarray, lam: float = LAMBDA_EST):
    """L_best of eq. (OurFinalLoss): lam (||Binf - Binf_hat||_1 + ||Bb - Bb_hat||_1) summed over the
    views, and its gradient w.r.t. the (V, 9) medium (B_d, B_b, B_inf); est is (V, 6) = (Binf_hat,
    Bb_hat)."""
    med = np.asarray(medium, np.float64).reshape(-1, 9)
    est = np.asarray(est, np.float64).reshape(-1, 6)
    d_inf = med[:, 6:9] - est[:, 0:3]
    d_b = med[:, 3:6] - est[:, 3:6]
    loss = lam * float(np.abs(d_inf).sum() + np.abs(d_b).sum())
    g = np.zeros_like(med)
    g[:, 6:9] = lam * np.sign(d_inf)
    g[:, 3:6] = lam * np.sign(d_b)
    return loss, g
