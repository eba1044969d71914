"""GPU parity of the fused L1 + D-SSIM loss pass (eq. 3DGSoriginalLoss, lambda 0.3) against the FP64
loss oracle: per-view losses and the gradient w.r.t. the rendered image, for ragged view sizes
(tiles cut by the image border on both axes), several views, lambda at its ends, and the rendered
image of the rasterizer as the prediction."""
import numpy as np
import pytest
import torch

from oracle import losses as LS
from paper_2411_19588_amd import rasterizer as R
from paper_2411_19588_amd import synth
from tests import gpu_util as U

pytestmark = pytest.mark.gpu


def _views(sizes):
    return [synth.Camera(w, h, float(w), float(w), w / 2.0, h / 2.0, np.eye(3, dtype=np.float32),
                         np.zeros(3, np.float32)) for w, h in sizes]


def _check(sizes, lam, seed, smooth=False):
    rng = np.random.default_rng(seed)
    cams = _views(sizes)
    rast = R.Rasterizer(cams)
    preds, tgts = [], []
    for w, h in sizes:
        t = rng.uniform(size=(3, h, w))
        p = np.clip(t + rng.normal(0, 0.1, size=(3, h, w)), 0, 1) if smooth else rng.uniform(size=(3, h, w))
        preds.append(p.astype(np.float32))
        tgts.append(t.astype(np.float32))
    pred = torch.from_numpy(np.concatenate([p.reshape(-1) for p in preds])).cuda()
    tgt = torch.from_numpy(np.concatenate([t.reshape(-1) for t in tgts])).cuda()
    loss, grad = R.l1_dssim_loss(pred, tgt, rast, lam)
    torch.cuda.synchronize()
    loss = loss.cpu().numpy().astype(np.float64)
    grad = grad.cpu().numpy().astype(np.float64)
    off = 0
    total = 0.0
    for v, (w, h) in enumerate(sizes):
        ref, gref = LS.l1_dssim(preds[v].astype(np.float64), tgts[v].astype(np.float64), lam)
        total += ref
        assert abs(loss[v] - ref) <= 2e-5 * max(1.0, abs(ref)), (v, loss[v], ref)
        g = grad[off: off + 3 * w * h].reshape(3, h, w)
        U.grad_close(g, gref, 1e-3, f"view {v} ({w}x{h}) gradient")
        off += 3 * w * h
    assert abs(loss[len(sizes)] - total) <= 2e-5 * max(1.0, total)
    U.say(f"  loss {sizes} lambda {lam}: total {loss[-1]:.6f} vs {total:.6f}")


@pytest.mark.parametrize("sizes", [[(32, 16)], [(45, 29)], [(7, 5)], [(203, 141)], [(96, 64), (33, 70), (130, 17)]])
def test_l1_dssim_vs_oracle(sizes):
    _check(sizes, 0.3, 5, smooth=True)


@pytest.mark.parametrize("lam", [0.0, 1.0])
def test_l1_dssim_lambda_ends(lam):
    _check([(70, 45)], lam, 6)


def test_l1_dssim_of_a_render(oracle_mod):
    """The rasterizer's image against a seeded target: the loss and its gradient as a training step sees them."""
    sc = synth.make_scene(1, n=5000, width=120, height=80)
    rast = U.make_rast(sc)
    rgb, depth, alpha, ctx, d = U.forward(sc, rast)
    tgt = torch.from_numpy(sc.targets[0].reshape(-1).astype(np.float32)).cuda()
    loss, grad = R.l1_dssim_loss(rgb, tgt, rast, 0.3)
    img = rgb.view(3, 80, 120).cpu().numpy().astype(np.float64)
    ref, gref = LS.l1_dssim(img, sc.targets[0].astype(np.float64), 0.3)
    assert abs(float(loss[0].item()) - ref) <= 2e-5
    U.grad_close(grad.view(3, 80, 120).cpu().numpy(), gref, 1e-3, "render gradient")
    # deterministic: a second call gives the same bits
    loss2, grad2 = R.l1_dssim_loss(rgb, tgt, rast, 0.3)
    assert torch.equal(loss, loss2) and torch.equal(grad, grad2)
