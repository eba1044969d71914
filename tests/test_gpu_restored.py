"""GPU parity of the restored outputs: the clean image J = C_air of eq. (scattering_approx), the
logistic depth image of the Implementation section, their adjoints, and the adjoint's use of the
cameras its forward saw."""
import numpy as np
import pytest
import torch

from paper_2411_19588_amd import rasterizer as R
from paper_2411_19588_amd import synth
from tests import gpu_util as U

pytestmark = pytest.mark.gpu

FIELDS = ("means", "scales", "quats", "opacity", "sh")


def _chw(a, cam):
    return torch.from_numpy(np.ascontiguousarray(a.T.reshape(3, cam.height, cam.width)).astype(np.float32))


@pytest.mark.parametrize("depth_mode,depth_output", [(0, 1), (1, 0), (1, 1)])
def test_restored_image_and_depth_image_vs_oracle(oracle_mod, depth_mode, depth_output):
    O = oracle_mod
    sc = synth.make_scene(1, n=8000, width=100, height=70)
    cam = sc.cameras[0]
    opts = O.Options(depth_mode=depth_mode, depth_output=depth_output)
    rast = U.make_rast(sc, depth_mode=depth_mode, depth_output=depth_output)
    d = U.to_dev(sc)
    rgb, depth, alpha, ctx = rast.forward(d["means"], d["scales"], d["quats"], d["opacity"], d["sh"], sc.sh_degree,
                                          d["medium"], restored=True)
    torch.cuda.synchronize()
    pix = U.pixel_list(cam.width, cam.height)
    orc = O.render(sc, cam, sc.medium[0], opts, pixels=pix, variants=4)
    n_main, n_var, worst = U.compare_pixels(*U.gather_view(rgb, depth, alpha, rast, 0, pix), orc)
    U.say(f"restored mode {depth_mode}/{depth_output}: main {n_main} variant {n_var} worst {worst:.2e}")
    J = ctx.restored.view(3, cam.height, cam.width).cpu().numpy()
    Jg = J[:, pix[:, 1], pix[:, 0]].T.astype(np.float64)
    clear = orc["nvar"] == 0
    err = np.abs(Jg - orc["cair"])[clear]
    U.say(f"  J: {int(clear.sum())} unambiguous pixels, worst {err.max():.2e}")
    assert err.max() <= U.IMG_TOL
    assert np.count_nonzero(orc["alpha"] > 0) > 1000
    # the same forward without the restored output renders the same image bits
    rgb2, depth2, alpha2, _ = rast.forward(d["means"], d["scales"], d["quats"], d["opacity"], d["sh"],
                                           sc.sh_degree, d["medium"])
    assert torch.equal(rgb, rgb2) and torch.equal(depth, depth2) and torch.equal(alpha, alpha2)


@pytest.mark.parametrize("depth_mode,depth_output", [(0, 0), (0, 1), (1, 1)])
def test_grad_with_restored_and_depth_upstream_vs_oracle(oracle_mod, depth_mode, depth_output):
    O = oracle_mod
    sc = synth.make_scene(1, n=3000, width=96, height=64)
    cam = sc.cameras[0]
    P = cam.width * cam.height
    rng = np.random.default_rng(17)
    G, GJ, Gz = rng.normal(size=(P, 3)), rng.normal(size=(P, 3)), rng.normal(size=P)
    opts = O.Options(depth_mode=depth_mode, depth_output=depth_output)
    G, Gz, n_amb = U.unambiguous(O, sc, 0, G, opts, Gz)
    GJ[G[:, 0] == 0] = 0.0
    U.say(f"grad with J and depth upstream, mode {depth_mode}/{depth_output}, ambiguous pixels {n_amb}")
    rast = U.make_rast(sc, depth_mode=depth_mode, depth_output=depth_output)
    rgb, depth, alpha, ctx, d = U.forward(sc, rast)
    out = rast.backward(ctx, d["means"], d["scales"], d["quats"], d["opacity"], d["sh"], d["medium"],
                        _chw(G, cam).reshape(-1).cuda(), torch.from_numpy(Gz.astype(np.float32)).cuda(),
                        grad_restored=_chw(GJ, cam).reshape(-1).cuda())
    torch.cuda.synchronize()
    got = dict(zip(FIELDS + ("medium",), [t.cpu().numpy().astype(np.float64) for t in out]))
    ref = O.backward(sc, cam, sc.medium[0], G, Gz, opts, grad_cair=GJ)
    for f in FIELDS:
        U.grad_close(got[f], ref[f], 1e-3, f)
    U.grad_close(got["medium"].reshape(-1), ref["medium"], 1e-3, "medium")


def test_autograd_restored_output(oracle_mod):
    """render(..., restored=True): gradients of a loss on C_uw and J through torch.autograd."""
    O = oracle_mod
    sc = synth.make_scene(1, n=2000, width=64, height=48)
    cam = sc.cameras[0]
    P = cam.width * cam.height
    rng = np.random.default_rng(23)
    G, GJ = rng.normal(size=(P, 3)), rng.normal(size=(P, 3))
    G, _, _ = U.unambiguous(O, sc, 0, G)
    GJ[G[:, 0] == 0] = 0.0
    rast = U.make_rast(sc)
    d = U.to_dev(sc)
    params = [d[k].clone().requires_grad_(True) for k in FIELDS + ("medium",)]
    rgb, depth, alpha, J = R.render(*params, rast, sc.sh_degree, restored=True)
    loss = (rgb * _chw(G, cam).reshape(-1).cuda()).sum() + (J * _chw(GJ, cam).reshape(-1).cuda()).sum()
    loss.backward()
    torch.cuda.synchronize()
    ref = O.backward(sc, cam, sc.medium[0], G, grad_cair=GJ)
    for f, p in zip(FIELDS, params):
        U.grad_close(p.grad.cpu().numpy().astype(np.float64), ref[f], 1e-3, f)
    U.grad_close(params[5].grad.cpu().numpy().reshape(-1).astype(np.float64), ref["medium"], 1e-3, "medium")


def test_backward_uses_the_cameras_of_its_forward(oracle_mod):
    """The poses change between forward and backward (set_cameras): the adjoint still pairs the saved
    records with the forward's cameras."""
    O = oracle_mod
    sc = synth.make_scene(1, n=3000, width=96, height=64)
    cam = sc.cameras[0]
    P = cam.width * cam.height
    G = np.random.default_rng(29).normal(size=(P, 3))
    G, _, _ = U.unambiguous(O, sc, 0, G)
    rast = U.make_rast(sc)
    rgb, depth, alpha, ctx, d = U.forward(sc, rast)
    moved = synth.look_at((0.4, -0.3, -0.2), (0.1, 0.2, 5.0), cam.width, cam.height)
    rast.set_cameras([moved])
    out = rast.backward(ctx, d["means"], d["scales"], d["quats"], d["opacity"], d["sh"], d["medium"],
                        _chw(G, cam).reshape(-1).cuda())
    torch.cuda.synchronize()
    ref = O.backward(sc, cam, sc.medium[0], G)
    for f, t in zip(FIELDS, out):
        U.grad_close(t.cpu().numpy().astype(np.float64), ref[f], 1e-3, f)
