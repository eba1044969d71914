"""Pins for the backscatter-estimation oracle (Alg. 1 and Alg. 2, L_best of eq. OurFinalLoss).

Known coefficients are recovered exactly from images whose darkest pixels follow the backscatter
model (a synthetic image, and a render of a scene whose Gaussians are all black, where the
underwater image is the backscatter alone); the clustering, the darkest-pixel selection, the
resize and the fit are checked against brute-force definitions written independently."""
import math

import numpy as np
import pytest

from oracle import backscatter as BS
from paper_2411_19588_amd import synth

TRUE_INF = np.array([0.2, 0.35, 0.5])
TRUE_B = np.array([0.8, 0.4, 1.5])


def _synthetic(w=200, h=150, seed=0, dark_frac=0.03):
    """Depth uniform in [1, 8]; a dark_frac share of the pixels is pure backscatter, the others add a
    direct signal of at least 0.3 per channel (so they are never among the darkest)."""
    rng = np.random.default_rng(seed)
    z = rng.uniform(1.0, 8.0, size=(h, w)).astype(np.float32)
    B = np.stack([BS.model(TRUE_INF[c], TRUE_B[c], z) for c in range(3)])
    sig = rng.uniform(0.3, 0.5, size=(3, h, w))
    dark = rng.uniform(size=(h, w)) < dark_frac
    I = np.where(dark[None], B, B + sig).astype(np.float32)
    return I, z, dark


def test_recovers_known_coefficients_from_synthetic_dark_pixels():
    I, z, dark = _synthetic()
    binf, bb, pts = BS.estimate(I, z, resize_height=0)
    for c in range(3):
        assert len(pts[c]) >= 9          # the darkest of a cluster sit at its near end
    np.testing.assert_allclose(binf, TRUE_INF, rtol=2e-6)
    np.testing.assert_allclose(bb, TRUE_B, rtol=2e-5)
    # the selection is exactly the dark pixels' darkest share, every one of them on the model
    sel = BS.dark_pixels(I, z)
    assert dark.reshape(-1)[sel].all()


def test_recovers_medium_from_a_render_of_a_black_scene(oracle_mod):
    """Every Gaussian black (colour 0): the underwater image is B_inf (1 - exp(-B_b z)) at the rendered
    depth z of eq. (Depth), so the estimate must return the medium the scene was rendered with."""
    O = oracle_mod
    sc = synth.custom_scene(seed=5, n=4000, sh_degree=0, width=160, height=120, lo=(-2.0, -1.5, 1.5),
                            hi=(2.0, 1.5, 9.0), log_scale_mean=-2.2)
    sc.sh[:] = np.float32(-math.sqrt(math.pi))        # 1/2 + Y00 k = 0: colour 0
    sc.opacity[:] = np.float32(0.95)
    med = np.array([0.3, 0.2, 0.1, *TRUE_B, *TRUE_INF])
    cam = sc.cameras[0]
    out = O.render(sc, cam, med)
    assert np.max(np.abs(out["cair"])) < 1e-7
    img = out["rgb"].reshape(cam.height, cam.width, 3).transpose(2, 0, 1).astype(np.float32)
    z = out["depth"].reshape(cam.height, cam.width).astype(np.float32)
    assert (z > 0).mean() > 0.9
    binf, bb, _ = BS.estimate(img, z, resize_height=0)
    np.testing.assert_allclose(binf, TRUE_INF, rtol=1e-5)
    np.testing.assert_allclose(bb, TRUE_B, rtol=1e-4)


def test_clusters_match_the_edges_definition_away_from_edges():
    rng = np.random.default_rng(1)
    z = rng.uniform(0.5, 9.5, size=5000).astype(np.float32)
    lo, hi = float(z.min()), float(z.max())
    got = BS._bins(z, lo, hi, 9)
    edges = np.linspace(lo, hi, 10)
    ref = np.clip(np.searchsorted(edges, z.astype(np.float64), side="right") - 1, 0, 8)
    near = np.min(np.abs(z[:, None].astype(np.float64) - edges[None, :]), axis=1) < 1e-5
    assert np.array_equal(got[~near], ref[~near])
    assert got.min() == 0 and got.max() == 8 and got[np.argmax(z)] == 8


def test_darkest_selection_matches_brute_force():
    rng = np.random.default_rng(2)
    h, w = 23, 31
    I = rng.uniform(size=(3, h, w)).astype(np.float32)
    I[:, 4, 5] = I[:, 9, 9]                          # a tie in the norm: the lower index comes first
    z = rng.uniform(1, 4, size=(h, w)).astype(np.float32)
    z[0, :5] = 0.0                                   # pixels without a depth take no part
    for p_dark in (0.01, 0.05, 0.3):
        got = BS.dark_pixels(I, z, p_dark)
        flat = [(k, float(z.reshape(-1)[k])) for k in range(h * w) if z.reshape(-1)[k] > 0]
        zs = np.array([f for _, f in flat], np.float32)
        cl = BS._bins(zs, zs.min(), zs.max(), 9)
        want = []
        for c in range(9):
            mem = [flat[i][0] for i in range(len(flat)) if cl[i] == c]
            if not mem:
                continue
            q = {k: (np.float32(I[0].reshape(-1)[k]) ** 2 + np.float32(I[1].reshape(-1)[k]) ** 2) +
                 np.float32(I[2].reshape(-1)[k]) ** 2 for k in mem}
            mem.sort(key=lambda k: (q[k], k))
            want += mem[:math.ceil(float(np.float32(p_dark)) * len(mem))]
        assert sorted(want) == list(got), p_dark


def test_resize_halving_averages_blocks():
    rng = np.random.default_rng(3)
    a = rng.uniform(size=(3, 8, 12)).astype(np.float32)
    r = BS.resize(a, 6, 4)
    ref = 0.25 * (a[:, 0::2, 0::2] + a[:, 0::2, 1::2] + a[:, 1::2, 0::2] + a[:, 1::2, 1::2])
    np.testing.assert_allclose(r, ref, rtol=1e-6)
    np.testing.assert_array_equal(BS.resize(a - 0.5, 12, 8), np.maximum(a - 0.5, 0))   # same size: clamp only
    assert BS.resized_size(1920, 1080, 300) == (533, 300)
    assert BS.resized_size(640, 480, 0) == (640, 480)


def test_fit_reaches_the_grid_minimum():
    """The bounded fit against a brute-force search: B_b on a fine grid, B_inf in closed form."""
    rng = np.random.default_rng(4)
    for trial in range(4):
        z = rng.uniform(0.5, 10.0, size=20)
        v = np.clip(BS.model(rng.uniform(0.05, 0.6), rng.uniform(0.1, 3.0), z) + rng.normal(0, 0.02, 20), 0, None)
        pts = list(zip(z, v))
        binf, bb = BS.fit(pts)
        assert 0 <= binf <= 1 and 0 <= bb <= 5
        grid = np.linspace(0.0, 5.0, 200001)
        f = 1.0 - np.exp(-grid[:, None] * z[None, :])
        a = np.clip((f * v).sum(1) / np.maximum((f * f).sum(1), 1e-300), 0.0, 1.0)
        res = ((a[:, None] * f - v) ** 2).sum(1)
        assert BS.residual(binf, bb, pts) <= res.min() * (1 + 1e-9) + 1e-15


def test_prior_loss_and_gradient():
    rng = np.random.default_rng(5)
    med = rng.uniform(0.05, 0.5, size=(3, 9))
    est = rng.uniform(0.05, 0.5, size=(3, 6))
    loss, g = BS.prior(med, est, 0.1)
    assert loss == pytest.approx(0.1 * (np.abs(med[:, 6:] - est[:, :3]).sum() + np.abs(med[:, 3:6] - est[:, 3:]).sum()))
    assert np.all(g[:, :3] == 0)
    h = 1e-7
    for v in range(3):
        for j in range(3, 9):
            mp, mm = med.copy(), med.copy()
            mp[v, j] += h
            mm[v, j] -= h
            fd = (BS.prior(mp, est, 0.1)[0] - BS.prior(mm, est, 0.1)[0]) / (2 * h)
            assert g[v, j] == pytest.approx(fd, abs=1e-7)
