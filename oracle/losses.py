"""Image losses of the training objective -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module.  It shares no code with the HIP library.

Sec. Optimization, eq. (3DGSoriginalLoss) and eq. (OurFinalLoss): the loss of one
rendered image I against its observation I_gt is

    (1 - lambda) * L1(I_gt, I) + lambda * L_D-SSIM(I_gt, I),    lambda = 0.3
    (appendix "Experimental Setup": Lambda SSIM),

summed over the K images of a batch.  The paper cites SSIM (Wang et al.) and
gives no window; the readings taken here are the SSIM literature's defaults:

* L1 = mean over the 3 H W values of |I - I_gt|;
* SSIM map per colour channel with an 11 x 11 Gaussian window of standard
  deviation 1.5 (normalised to sum 1), "same" size with zero padding outside
  the image, C1 = (0.01)^2, C2 = (0.03)^2 (dynamic range 1):

      mu_x = w * x,  sigma_x^2 = w * x^2 - mu_x^2,  sigma_xy = w * (x y) - mu_x mu_y
      S = (2 mu_x mu_y + C1)(2 sigma_xy + C2) / ((mu_x^2 + mu_y^2 + C1)(sigma_x^2 + sigma_y^2 + C2));

* L_D-SSIM = 1 - mean of S over the 3 H W values.

Everything is FP64.  The window sums are a library 2D correlation
(``scipy.ndimage.correlate``, constant zero padding); the gradient is the exact
derivative of the definition above, written out.
"""
from __future__ import annotations

import numpy as np
from scipy import ndimage

WINDOW = 11
SIGMA = 1.5
C1 = 0.01 ** 2
C2 = 0.03 ** 2
LAMBDA_SSIM = 0.3


def gaussian_window(size: int = WINDOW, sigma: float = SIGMA) -> np.ndarray:
    """The 2D window: outer product of the normalised 1D Gaussian (sums to 1)."""
    r = np.arange(size, dtype=np.float64) - (size - 1) / 2.0
    g = np.exp(-(r * r) / (2.0 * sigma * sigma))
    g /= g.sum()
    return np.outer(g, g)


def _blur(a: np.ndarray, w: np.ndarray) -> np.ndarray:
    """Windowed sum around every pixel of a 2D map, zero outside the image."""
    return ndimage.correlate(np.asarray(a, np.float64), w, mode="constant", cval=0.0)


def ssim_map(x: np.ndarray, y: np.ndarray, w: np.ndarray = None):
    """SSIM map of one channel (H, W) and the intermediate terms."""
    w = gaussian_window() if w is None else w
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    mx, my = _blur(x, w), _blur(y, w)
    sxx = _blur(x * x, w) - mx * mx
    syy = _blur(y * y, w) - my * my
    sxy = _blur(x * y, w) - mx * my
    A1 = 2.0 * mx * my + C1
    A2 = 2.0 * sxy + C2
    B1 = mx * mx + my * my + C1
    B2 = sxx + syy + C2
    return A1 * A2 / (B1 * B2), dict(mx=mx, my=my, A1=A1, A2=A2, B1=B1, B2=B2)


def dssim(pred: np.ndarray, target: np.ndarray) -> float:
    """1 - mean SSIM over the channels and pixels of a (3, H, W) image."""
    return 1.0 - float(np.mean([ssim_map(pred[c], target[c])[0] for c in range(pred.shape[0])]))


def dssim_grad(pred: np.ndarray, target: np.ndarray) -> np.ndarray:
    """d(1 - mean S)/d pred, (3, H, W).

    With m1 = w * x, m2 = w * x^2 and m12 = w * (x y) at each pixel p, S depends on x only
    through them, so  dS(p)/dx(q) = w(q - p) [dS/dm1 + 2 x(q) dS/dm2 + y(q) dS/dm12](p),
    and the windowed sums back to q are the adjoint of the zero-padded correlation (the window
    is symmetric, so it is the same correlation restricted to the image).
    """
    w = gaussian_window()
    C, H, W = pred.shape
    g = np.zeros((C, H, W))
    scale = -1.0 / (C * H * W)                 # d(1 - mean S)/dS(p)
    for c in range(C):
        x = np.asarray(pred[c], np.float64)
        y = np.asarray(target[c], np.float64)
        S, t = ssim_map(x, y, w)
        mx, my, A1, A2, B1, B2 = t["mx"], t["my"], t["A1"], t["A2"], t["B1"], t["B2"]
        den = B1 * B2
        # partial derivatives of S w.r.t. (m1, m2, m12), with sigma_x^2 = m2 - m1^2 and
        # sigma_xy = m12 - m1 mu_y
        dA1 = 2.0 * my
        dA2 = -2.0 * my
        dB1 = 2.0 * mx
        dB2 = -2.0 * mx
        dS_dm1 = (dA1 * A2 + A1 * dA2) / den - S * (dB1 / B1 + dB2 / B2)
        dS_dm2 = -S / B2
        dS_dm12 = 2.0 * A1 / den
        a = _blur(scale * dS_dm1, w)
        b = _blur(scale * dS_dm2, w)
        d = _blur(scale * dS_dm12, w)
        g[c] = a + 2.0 * x * b + y * d
    return g


def l1(pred: np.ndarray, target: np.ndarray):
    """Mean absolute error and its gradient sign(pred - target) / numel."""
    d = np.asarray(pred, np.float64) - np.asarray(target, np.float64)
    return float(np.mean(np.abs(d))), np.sign(d) / d.size


def l1_dssim(pred: np.ndarray, target: np.ndarray, lam: float = LAMBDA_SSIM):
    """(1 - lambda) L1 + lambda D-SSIM of one (3, H, W) image and its gradient w.r.t. pred."""
    l, gl = l1(pred, target)
    return (1.0 - lam) * l + lam * dssim(pred, target), (1.0 - lam) * gl + lam * dssim_grad(pred, target)


def l1_dssim_views(preds, targets, lam: float = LAMBDA_SSIM):
    """Sum over the views of the per-view loss (eq. 3DGSoriginalLoss sums over the K images)."""
    tot, grads = 0.0, []
    for p, t in zip(preds, targets):
        v, g = l1_dssim(p, t, lam)
        tot += v
        grads.append(g)
    return tot, grads
