"""Parity at full size, in the launch configurations the benchmark times: sampled pixels of every
image against the FP64 oracle, and gradients of a loss on a 64x64 crop for 200 sampled Gaussians
against the oracle's exact gradient (and FP64 central differences for every parameter of the
crop's most influential Gaussians), for the 300k-Gaussian 1600x1067 training workload, the
1M-Gaussian 1920x1080 workload, the 24-view batched workload and the 3M-Gaussian 4-view
workload; and the first moments of one full-scale fused training step."""
import numpy as np
import pytest
import torch

from paper_2411_19588_amd import rasterizer as R
from paper_2411_19588_amd import synth
from tests import gpu_util as U

pytestmark = pytest.mark.gpu

FIELDS = ("means", "scales", "quats", "opacity", "sh")
CROP = (912, 500, 64, 64)          # x0, y0, width, height


@pytest.fixture(scope="module")
def scene():
    return synth.make_scene(2)


def _bench_rast(sc):
    return R.Rasterizer(sc.cameras, R.RasterConfig())    # the benchmark's default launch configuration


def test_image_full_size_sampled(oracle_mod, scene):
    O = oracle_mod
    sc = scene
    cam = sc.cameras[0]
    rast = _bench_rast(sc)
    rgb, depth, alpha, ctx, _ = U.forward(sc, rast)
    st, _ = rast.read_status(ctx.saved)
    assert st == 0
    rng = np.random.default_rng(11)
    pix = np.stack([rng.integers(0, cam.width, 6000), rng.integers(0, cam.height, 6000)], 1)
    # plus the ragged last tile row and the frame corners
    edge = np.stack([rng.integers(0, cam.width, 500), rng.integers(cam.height - 8, cam.height, 500)], 1)
    corners = np.array([[0, 0], [cam.width - 1, 0], [0, cam.height - 1], [cam.width - 1, cam.height - 1]])
    pix = np.ascontiguousarray(np.concatenate([pix, edge, corners]).astype(np.int32))
    U.say(f"full-size image, {len(pix)} sampled pixels")
    orc = O.render(sc, cam, sc.medium[0], pixels=pix, variants=4)
    n_main, n_var, worst = U.compare_pixels(*U.gather_view(rgb, depth, alpha, rast, 0, pix), orc)
    U.say(f"  main {n_main} variant {n_var} worst {worst:.2e}")


def test_image_full_size_24_views_sampled(oracle_mod):
    """The batched workload at full size (1M Gaussians, 24 views of uneven resolution, 29.5 Mpixel)
    in the launch configuration the autotuner picks for it: 250 random pixels and the four corners
    of every view against the FP64 oracle."""
    O = oracle_mod
    sc = synth.make_scene(3)
    rast = R.Rasterizer(sc.cameras, R.RasterConfig(tile=16, pixels_per_lane=4, record_fetch="scalar",
                                                   lds_batch=256, persistent=False, phases=4, phase0_shift=6))
    rgb, depth, alpha, ctx, _ = U.forward(sc, rast)
    st, _ = rast.read_status(ctx.saved)
    assert st == 0
    rng = np.random.default_rng(12)
    U.say(f"full-size 24 views, {len(sc.cameras)} x 254 sampled pixels")
    for v, cam in enumerate(sc.cameras):
        pix = np.stack([rng.integers(0, cam.width, 250), rng.integers(0, cam.height, 250)], 1)
        corners = np.array([[0, 0], [cam.width - 1, 0], [0, cam.height - 1], [cam.width - 1, cam.height - 1]])
        pix = np.ascontiguousarray(np.concatenate([pix, corners]).astype(np.int32))
        orc = O.render(sc, cam, sc.medium[v], pixels=pix, variants=4)
        U.compare_pixels(*U.gather_view(rgb, depth, alpha, rast, v, pix), orc)


def test_image_full_size_3m_4_views_sampled(oracle_mod):
    """The full-scale training workload's forward (3M Gaussians SH 3, 4 views at 1920x1080) in the
    default launch configuration and automatic several-view schedule: 250 random pixels, the four
    corners and the ragged last tile row of every view against the FP64 oracle."""
    O = oracle_mod
    sc = synth.make_scene(4)
    rast = R.Rasterizer(sc.cameras, R.RasterConfig())
    rgb, depth, alpha, ctx, _ = U.forward(sc, rast)
    st, _ = rast.read_status(ctx.saved)
    assert st == 0
    rng = np.random.default_rng(13)
    U.say(f"full-size 3M Gaussians, {len(sc.cameras)} views x 270 sampled pixels, schedule {rast.schedule(sc.n)}")
    for v, cam in enumerate(sc.cameras):
        pix = np.stack([rng.integers(0, cam.width, 250), rng.integers(0, cam.height, 250)], 1)
        corners = np.array([[0, 0], [cam.width - 1, 0], [0, cam.height - 1], [cam.width - 1, cam.height - 1]])
        last_row = np.stack([rng.integers(0, cam.width, 16), np.full(16, cam.height - 1)], 1)
        pix = np.ascontiguousarray(np.concatenate([pix, corners, last_row]).astype(np.int32))
        orc = O.render(sc, cam, sc.medium[v], pixels=pix, variants=4)
        U.compare_pixels(*U.gather_view(rgb, depth, alpha, rast, v, pix), orc)


AUTOTUNED_24 = dict(tile=16, pixels_per_lane=4, record_fetch="scalar", lds_batch=256, persistent=False, phases=4,
                   phase0_shift=6)


def test_image_full_size_config1_sampled(oracle_mod):
    """The 300k-Gaussian training workload (SH 3, one 1600x1067 view) in the default launch
    configuration and automatic schedule: 6,000 random pixels, the ragged last tile row (1067 = 66 x 16
    + 11) and the corners against the FP64 oracle."""
    O = oracle_mod
    sc = synth.make_scene(1)
    cam = sc.cameras[0]
    rast = R.Rasterizer(sc.cameras, R.RasterConfig())
    rgb, depth, alpha, ctx, _ = U.forward(sc, rast)
    st, _ = rast.read_status(ctx.saved)
    assert st == 0
    rng = np.random.default_rng(15)
    pix = np.stack([rng.integers(0, cam.width, 6000), rng.integers(0, cam.height, 6000)], 1)
    edge = np.stack([rng.integers(0, cam.width, 500), rng.integers(cam.height - 11, cam.height, 500)], 1)
    corners = np.array([[0, 0], [cam.width - 1, 0], [0, cam.height - 1], [cam.width - 1, cam.height - 1]])
    pix = np.ascontiguousarray(np.concatenate([pix, edge, corners]).astype(np.int32))
    U.say(f"full-size 300k Gaussians 1600x1067, {len(pix)} sampled pixels, schedule {rast.schedule(sc.n)}")
    orc = O.render(sc, cam, sc.medium[0], pixels=pix, variants=4)
    U.compare_pixels(*U.gather_view(rgb, depth, alpha, rast, 0, pix), orc)


@pytest.mark.timeout(600)
def test_grad_full_size_crop(oracle_mod, scene):
    """1M Gaussians, 1920x1080, the benchmark's launch configuration: the crop gradient for 200 sampled
    Gaussians, and central differences of all 59 parameters of the 20 Gaussians with the largest
    opacity gradient."""
    O = oracle_mod
    sc = scene
    U.say("full-size crop gradient, 1M Gaussians 1920x1080")
    got, ref, Gc, pix, live = U.crop_grad_check(O, sc, _bench_rast(sc), 0, CROP, 12)
    U.fd_crop_check(O, sc, 0, CROP, Gc, got, ref, live, 20)


@pytest.mark.timeout(600)
def test_grad_full_size_config1_crop(oracle_mod):
    """300k Gaussians, 1600x1067: the crop gradient (a crop reaching into the ragged last tile row) for 200
    sampled Gaussians, and central differences of every parameter of 10 of them."""
    O = oracle_mod
    sc = synth.make_scene(1)
    crop = (760, 1067 - 64, 64, 64)
    U.say("full-size crop gradient, 300k Gaussians 1600x1067")
    got, ref, Gc, pix, live = U.crop_grad_check(O, sc, R.Rasterizer(sc.cameras, R.RasterConfig()), 0, crop, 16)
    U.fd_crop_check(O, sc, 0, crop, Gc, got, ref, live, 10)


def test_grad_full_size_crop_24_views(oracle_mod):
    """The batched workload (1M Gaussians, 24 views of uneven resolution) in the autotuner's launch
    configuration: the crop gradient on one 1920x1080 view, zero upstream gradient in the other 23."""
    O = oracle_mod
    sc = synth.make_scene(3)
    v = next(i for i, c in enumerate(sc.cameras) if (c.width, c.height) == (1920, 1080))
    U.say(f"full-size 24-view crop gradient (view {v})")
    U.crop_grad_check(O, sc, R.Rasterizer(sc.cameras, R.RasterConfig(**AUTOTUNED_24)), v, CROP, 18)


def test_grad_full_size_crop_4_views(oracle_mod):
    """The 3M-Gaussian, 4-view workload (default launch configuration, automatic schedule): the
    gradient of a loss on a 64x64 crop of view 1, zero upstream gradient elsewhere and in the other
    views, through the several-view adjoint (the SH part in k_sh_views), against the oracle's exact
    gradient for 200 sampled Gaussians; each view's medium gradient (zero but for view 1)."""
    O = oracle_mod
    sc = synth.make_scene(4)
    U.say("full-size 4-view crop gradient (view 1)")
    U.crop_grad_check(O, sc, R.Rasterizer(sc.cameras, R.RasterConfig()), 1, CROP, 14)


def test_fused_training_step_full_size_3m_4_views_first_moments(oracle_mod):
    """One step of the full-scale training workload (3M Gaussians SH 3, 4 views at 1920x1080, Adam fused
    into the adjoint, as the benchmark trains): the first moments m = (1 - beta1) g of every group against
    the oracle's gradient of the L1 loss, with the target equal to the rendered image outside a 64x64
    crop of view 2."""
    from paper_2411_19588_amd.trainer import TrainStep
    O = oracle_mod
    sc = synth.make_scene(4)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a))
    ts = TrainStep(t(sc.means), t(sc.log_scales), t(sc.quats), t(sc.logits), t(sc.sh), t(sc.medium),
                   sc.sh_degree, sc.cameras, torch.cat([t(x).reshape(-1) for x in sc.targets]), R.RasterConfig(),
                   fused=True)
    ts.size_capacity()
    U.say("full-size fused training step, first moments vs oracle (view 2)")
    U.first_moment_check(O, sc, ts, 2, CROP, torch.cuda.Stream())
