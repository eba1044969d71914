"""Pins for the loss oracle (L1 + D-SSIM of eq. 3DGSoriginalLoss / OurFinalLoss).

The window sums are checked against explicit windowed sums written as loops (zero padding,
orientation), the SSIM map against its closed forms (identical images give 1, constant images
give the luminance term), and the gradient against FP64 central differences."""
import math

import numpy as np
import pytest

from oracle import losses as LS


def test_window_is_a_normalised_separable_gaussian():
    w = LS.gaussian_window()
    assert w.shape == (11, 11)
    assert w.sum() == pytest.approx(1.0, abs=1e-15)
    np.testing.assert_allclose(w, w.T, rtol=0, atol=0)
    np.testing.assert_allclose(w, w[::-1, ::-1], rtol=0, atol=0)
    # ratio of neighbouring taps of a Gaussian of standard deviation 1.5
    for k in range(1, 6):
        r = w[5, 5 + k] / w[5, 5 + k - 1]
        assert r == pytest.approx(math.exp(-((k * k) - (k - 1) ** 2) / (2 * 1.5 ** 2)), rel=1e-13)
    u, s, vt = np.linalg.svd(w)
    assert s[1] < 1e-15 * s[0]          # rank one: separable


def _brute_moments(x, y, w):
    """Windowed sums around every pixel by explicit loops, zero outside the image."""
    H, W = x.shape
    r = w.shape[0] // 2
    out = np.zeros((5, H, W))
    for i in range(H):
        for j in range(W):
            acc = np.zeros(5)
            for di in range(-r, r + 1):
                for dj in range(-r, r + 1):
                    ii, jj = i + di, j + dj
                    if 0 <= ii < H and 0 <= jj < W:
                        wt = w[di + r, dj + r]
                        a, b = x[ii, jj], y[ii, jj]
                        acc += wt * np.array([a, b, a * a, b * b, a * b])
            out[:, i, j] = acc
    return out


def test_ssim_map_matches_explicit_window_sums():
    rng = np.random.default_rng(0)
    x, y = rng.uniform(size=(9, 13)), rng.uniform(size=(9, 13))
    w = LS.gaussian_window()
    mx, my, mxx, myy, mxy = _brute_moments(x, y, w)
    sxx, syy, sxy = mxx - mx * mx, myy - my * my, mxy - mx * my
    ref = ((2 * mx * my + LS.C1) * (2 * sxy + LS.C2)) / ((mx * mx + my * my + LS.C1) * (sxx + syy + LS.C2))
    S, _ = LS.ssim_map(x, y)
    np.testing.assert_allclose(S, ref, rtol=1e-12, atol=1e-14)
    # asymmetric window contents: a single bright pixel's window sum lands on its neighbours
    z = np.zeros((15, 15))
    z[3, 10] = 1.0
    m = LS._blur(z, w)
    assert m[3, 10] == pytest.approx(w[5, 5])
    assert m[5, 9] == pytest.approx(w[5 - 2, 5 + 1])
    assert m[3 + 6, 10] == 0.0


def test_identical_images_give_one_and_zero_gradient():
    rng = np.random.default_rng(1)
    x = rng.uniform(size=(3, 20, 17))
    for c in range(3):
        S, _ = LS.ssim_map(x[c], x[c])
        np.testing.assert_allclose(S, 1.0, rtol=0, atol=1e-14)
    assert LS.dssim(x, x) == pytest.approx(0.0, abs=1e-14)
    np.testing.assert_allclose(LS.dssim_grad(x, x), 0.0, atol=1e-14)


def test_constant_images_interior_closed_form():
    a, b = 0.3, 0.7
    x, y = np.full((24, 24), a), np.full((24, 24), b)
    S, _ = LS.ssim_map(x, y)
    inner = S[5:-5, 5:-5]          # windows entirely inside the image
    np.testing.assert_allclose(inner, (2 * a * b + LS.C1) / (a * a + b * b + LS.C1), rtol=1e-12)
    assert not np.allclose(S[0, 0], inner[0, 0])   # the zero padding changes the border


def test_ssim_symmetric_in_its_arguments():
    rng = np.random.default_rng(2)
    x, y = rng.uniform(size=(11, 19)), rng.uniform(size=(11, 19))
    np.testing.assert_allclose(LS.ssim_map(x, y)[0], LS.ssim_map(y, x)[0], rtol=1e-13)


@pytest.mark.parametrize("shape", [(3, 12, 15), (3, 7, 23)])
def test_dssim_gradient_matches_central_differences(shape):
    rng = np.random.default_rng(3)
    x, y = rng.uniform(size=shape), rng.uniform(size=shape)
    g = LS.dssim_grad(x, y)
    h = 1e-6
    idx = [tuple(rng.integers(0, s) for s in shape) for _ in range(40)] + [(0, 0, 0), (2, shape[1] - 1, shape[2] - 1)]
    for i in idx:
        xp, xm = x.copy(), x.copy()
        xp[i] += h
        xm[i] -= h
        fd = (LS.dssim(xp, y) - LS.dssim(xm, y)) / (2 * h)
        assert abs(g[i] - fd) <= 1e-7 * max(1.0, abs(fd)) + 1e-9, (i, g[i], fd)


def test_l1_dssim_combination():
    rng = np.random.default_rng(4)
    x, y = rng.uniform(size=(3, 10, 12)), rng.uniform(size=(3, 10, 12))
    v, g = LS.l1_dssim(x, y, 0.3)
    assert v == pytest.approx(0.7 * np.mean(np.abs(x - y)) + 0.3 * LS.dssim(x, y), rel=1e-14)
    np.testing.assert_allclose(g, 0.7 * np.sign(x - y) / x.size + 0.3 * LS.dssim_grad(x, y), rtol=1e-14)
    # lambda = 0 is the L1 term alone
    v0, g0 = LS.l1_dssim(x, y, 0.0)
    assert v0 == pytest.approx(np.mean(np.abs(x - y)), rel=1e-15)
    tot, grads = LS.l1_dssim_views([x, y], [y, x], 0.3)
    assert tot == pytest.approx(2 * v, rel=1e-13)   # SSIM and L1 are symmetric in the two images
