"""GPU parity of the adjoint: gradients vs the FP64 oracle gradient and FP64 central differences."""
import dataclasses

import numpy as np
import pytest
import torch

from paper_2411_19588_amd import rasterizer as R
from paper_2411_19588_amd import synth
from paper_2411_19588_amd import _native as N
from tests import gpu_util as U

pytestmark = pytest.mark.gpu

FIELDS = ("means", "scales", "quats", "opacity", "sh")


def _gpu_grads(scene, rast, G, Gz=None):
    """Backward of L = <G, rgb> + <Gz, depth> for view 0 (G is (P,3) row-major pixels)."""
    rgb, depth, alpha, ctx, d = U.forward(scene, rast)
    cam = scene.cameras[0]
    g_rgb = torch.from_numpy(np.ascontiguousarray(G.T.reshape(3, cam.height, cam.width)).astype(np.float32))
    g_rgb = g_rgb.reshape(-1).cuda()
    g_dep = None if Gz is None else torch.from_numpy(Gz.astype(np.float32)).cuda()
    out = rast.backward(ctx, d["means"], d["scales"], d["quats"], d["opacity"], d["sh"], d["medium"], g_rgb, g_dep)
    torch.cuda.synchronize()
    return dict(zip(FIELDS + ("medium",), [t.cpu().numpy().astype(np.float64) for t in out]))


def _check_all(got, ref, rel=1e-3):
    for f in FIELDS:
        U.grad_close(got[f], ref[f], rel, f)
    U.grad_close(got["medium"].reshape(-1), ref["medium"], rel, "medium")


@pytest.mark.parametrize("depth_mode,with_gz", [(0, False), (0, True), (1, True)])
def test_grad_vs_oracle_small(oracle_mod, depth_mode, with_gz):
    O = oracle_mod
    sc = synth.make_scene(1, n=3000, width=96, height=64)
    cam = sc.cameras[0]
    P = cam.width * cam.height
    rng = np.random.default_rng(7)
    G = rng.normal(size=(P, 3))
    Gz = rng.normal(size=P) if with_gz else None
    G, Gz, n_amb = U.unambiguous(O, sc, 0, G, O.Options(depth_mode=depth_mode), Gz)
    U.say(f"grad small mode {depth_mode} gz {with_gz} ambiguous pixels {n_amb}")
    got = _gpu_grads(sc, U.make_rast(sc, depth_mode=depth_mode), G, Gz)
    ref = O.backward(sc, cam, sc.medium[0], G, Gz, O.Options(depth_mode=depth_mode))
    _check_all(got, ref)


def test_grad_vs_oracle_sh_degree0_config0(oracle_mod):
    O = oracle_mod
    sc = synth.make_scene(0)
    cam = sc.cameras[0]
    G = np.random.default_rng(8).normal(size=(cam.width * cam.height, 3))
    G, _, n_amb = U.unambiguous(O, sc, 0, G)
    U.say(f"grad config0 ambiguous pixels {n_amb}")
    got = _gpu_grads(sc, U.make_rast(sc), G)
    _check_all(got, O.backward(sc, cam, sc.medium[0], G))


def test_grad_vs_oracle_opacity_edge_values(oracle_mod):
    """Opacities of 0, below 0, 1e-30 and 1 mixed in: the adjoint forms the opacity term as
    (sum of dalpha * raw alpha) / o from the record's 1/o, which is 0 for o <= 0."""
    O = oracle_mod
    sc = synth.make_scene(0)
    op = sc.opacity.copy()
    op[0::7] = 0.0
    op[1::7] = -0.25
    op[2::7] = 1e-30
    op[3::7] = 1.0
    sc = dataclasses.replace(sc, opacity=op)
    cam = sc.cameras[0]
    G = np.random.default_rng(11).normal(size=(cam.width * cam.height, 3))
    G, _, n_amb = U.unambiguous(O, sc, 0, G)
    U.say(f"grad edge opacities, ambiguous pixels {n_amb}")
    got = _gpu_grads(sc, U.make_rast(sc), G)
    _check_all(got, O.backward(sc, cam, sc.medium[0], G))
    assert np.all(got["opacity"][0::7] == 0.0) and np.all(got["opacity"][1::7] == 0.0)


@pytest.mark.parametrize("cfg", [dict(lds_batch=256), dict(persistent=True), dict(tile=8, lds_batch=64),
                                 dict(record_fetch="lds"), dict(record_fetch="lds", pixels_per_lane=2, lds_batch=128),
                                 dict(record_fetch="lds", pixels_per_lane=4, persistent=True),
                                 dict(pixels_per_lane=1), dict(pixels_per_lane=4),
                                 dict(pixels_per_lane=1, persistent=True, lds_batch=64),
                                 dict(record_fetch="scalar", pixels_per_lane=1),
                                 dict(record_fetch="scalar", pixels_per_lane=2, persistent=True),
                                 dict(record_fetch="scalar", pixels_per_lane=4),
                                 dict(tile=8, lds_batch=64, record_fetch="scalar", persistent=True),
                                 dict(persistent=2), dict(persistent=2, record_fetch="lds", pixels_per_lane=2),
                                 dict(persistent=2, phases=3, phase0_shift=5)])
def test_grad_launch_variants(oracle_mod, cfg):
    O = oracle_mod
    sc = synth.make_scene(1, n=3000, width=96, height=64)
    cam = sc.cameras[0]
    G = np.random.default_rng(9).normal(size=(cam.width * cam.height, 3))
    G, _, _ = U.unambiguous(O, sc, 0, G)
    U.say(f"grad variant {cfg}")
    got = _gpu_grads(sc, U.make_rast(sc, **cfg), G)
    _check_all(got, O.backward(sc, cam, sc.medium[0], G))


def test_grad_vs_central_differences(oracle_mod):
    """GPU gradient vs FP64 central differences of the oracle forward on a tiny scene."""
    O = oracle_mod
    sc = synth.custom_scene(seed=21, n=30, sh_degree=3, width=32, height=24, f=36.0, log_scale_mean=-2.0,
                            sh_std=0.3)
    cam = sc.cameras[0]
    rng = np.random.default_rng(1)
    G = rng.normal(size=(cam.width * cam.height, 3))
    U.say("grad vs FD")
    got = _gpu_grads(sc, U.make_rast(sc), G)
    med = sc.medium[0].astype(np.float64)
    live = np.nonzero(np.abs(got["opacity"]) > 0)[0][:10]
    checked = 0
    for g in live:
        for f, rows in (("means", 3), ("scales", 3), ("quats", 4), ("opacity", 0), ("sh", 6)):
            for r in (range(rows) if rows else [None]):
                idx = (g,) if r is None else (r, g)
                fd, ok = O.fd_grad(sc, cam, med, G, f, idx)
                if not ok:
                    continue
                scale = np.sqrt(np.mean(got[f] ** 2))
                assert abs(got[f][idx] - fd) <= 1e-3 * abs(fd) + 1e-3 * scale, (f, idx, got[f][idx], fd)
                checked += 1
    for j in range(9):
        fd, ok = O.fd_grad(sc, cam, med, G, "medium", j)
        if ok:
            assert abs(got["medium"].reshape(-1)[j] - fd) <= 1e-3 * abs(fd) + 1e-6
            checked += 1
    assert checked > 80


def test_autograd_function_and_activation(oracle_mod):
    O = oracle_mod
    sc = synth.make_scene(1, n=2000, width=80, height=60)
    cam = sc.cameras[0]
    rast = U.make_rast(sc)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda().requires_grad_(True)
    ls, lg = t(sc.log_scales), t(sc.logits)
    means, quats, sh, med = t(sc.means), t(sc.quats), t(sc.sh), t(sc.medium)
    scales, opacity = R.activate(ls, lg)
    rgb, depth, alpha = R.render(means, scales, quats, opacity, sh, med, rast, sc.sh_degree)
    G = np.random.default_rng(3).normal(size=(cam.width * cam.height, 3))
    G, _, _ = U.unambiguous(O, sc, 0, G)
    Gt = torch.from_numpy(G.T.reshape(-1).astype(np.float32)).cuda()
    (rgb * Gt).sum().backward()
    U.say("autograd")
    # oracle on the activated values the GPU used
    s_dev = scales.detach().cpu().numpy()
    o_dev = opacity.detach().cpu().numpy()
    s_ref, o_ref = O.activate(sc.log_scales, sc.logits)
    np.testing.assert_allclose(s_dev, s_ref, rtol=2e-6)
    np.testing.assert_allclose(o_dev, o_ref, rtol=2e-6)
    sc2 = synth.Scene(**{**sc.__dict__, "scales": s_dev, "opacity": o_dev})
    ref = O.backward(sc2, cam, sc.medium[0], G)
    U.grad_close(means.grad.cpu().numpy(), ref["means"], 1e-3, "means")
    U.grad_close(ls.grad.cpu().numpy(), ref["scales"] * s_dev, 1e-3, "log_scales")
    U.grad_close(lg.grad.cpu().numpy(), ref["opacity"] * o_dev * (1 - o_dev), 1e-3, "logits")
    U.grad_close(quats.grad.cpu().numpy(), ref["quats"], 1e-3, "quats")
    U.grad_close(sh.grad.cpu().numpy(), ref["sh"], 1e-3, "sh")
    U.grad_close(med.grad.cpu().numpy().reshape(-1), ref["medium"], 1e-3, "medium")


@pytest.mark.parametrize("n,deg", [(2000, 3), (2001, 3), (1000, 2), (1001, 1), (1000, 0)])
def test_multiview_grad_sums_views(oracle_mod, n, deg):
    """Several views: the gradients are the sums of the views' oracle gradients (the SH part and the
    means' SH term come from k_sh_views; odd n takes its one-Gaussian-per-lane form).  Lower SH
    degrees keep the first (deg + 1)^2 coefficients of the degree-3 scene."""
    O = oracle_mod
    sc = synth.make_scene(3, n=n, n_views=3, view_sizes=[(64, 48), (80, 40), (48, 48)])
    if deg < 3:
        sc = dataclasses.replace(sc, sh=np.ascontiguousarray(sc.sh[:3 * (deg + 1) ** 2]), sh_degree=deg)
    rast = U.make_rast(sc)
    rgb, depth, alpha, ctx, d = U.forward(sc, rast)
    rng = np.random.default_rng(5)
    Gs = [U.unambiguous(O, sc, v, rng.normal(size=(c.width * c.height, 3)))[0] for v, c in enumerate(sc.cameras)]
    g_rgb = torch.cat([torch.from_numpy(G.T.reshape(-1).astype(np.float32)) for G in Gs]).cuda()
    out = rast.backward(ctx, d["means"], d["scales"], d["quats"], d["opacity"], d["sh"], d["medium"], g_rgb)
    got = dict(zip(FIELDS + ("medium",), [t.cpu().numpy().astype(np.float64) for t in out]))
    U.say(f"multiview grad n={n} sh degree {deg}")
    ref = {f: 0.0 for f in FIELDS}
    for v, cam in enumerate(sc.cameras):
        r = O.backward(sc, cam, sc.medium[v], Gs[v])
        for f in FIELDS:
            ref[f] = ref[f] + r[f]
        U.grad_close(got["medium"][v], r["medium"], 1e-3, f"medium view {v}")
    for f in FIELDS:
        U.grad_close(got[f], ref[f], 1e-3, f)


def test_multiview_grad_max_views(oracle_mod):
    """GS_MAX_VIEWS views: the gradients (k_sh_views with 3 + 3 * 64 planes) are the sums of the
    views' oracle gradients, and each view's medium gradient is its own."""
    O = oracle_mod
    V = N.GS_MAX_VIEWS
    sizes = [(16 + 8 * (v % 3), 16 + 8 * (v % 2)) for v in range(V)]
    sc = synth.make_scene(3, n=600, n_views=V, view_sizes=sizes)
    rast = U.make_rast(sc)
    rgb, depth, alpha, ctx, d = U.forward(sc, rast)
    rng = np.random.default_rng(9)
    Gs = [U.unambiguous(O, sc, v, rng.normal(size=(c.width * c.height, 3)))[0] for v, c in enumerate(sc.cameras)]
    g_rgb = torch.cat([torch.from_numpy(G.T.reshape(-1).astype(np.float32)) for G in Gs]).cuda()
    out = rast.backward(ctx, d["means"], d["scales"], d["quats"], d["opacity"], d["sh"], d["medium"], g_rgb)
    got = dict(zip(FIELDS + ("medium",), [t.cpu().numpy().astype(np.float64) for t in out]))
    U.say(f"multiview grad {V} views")
    ref = {f: 0.0 for f in FIELDS}
    for v, cam in enumerate(sc.cameras):
        r = O.backward(sc, cam, sc.medium[v], Gs[v])
        for f in FIELDS:
            ref[f] = ref[f] + r[f]
        U.grad_close(got["medium"][v], r["medium"], 1e-3, f"medium view {v}")
    for f in FIELDS:
        U.grad_close(got[f], ref[f], 1e-3, f)


def test_l1_loss_and_adam(oracle_mod):
    O = oracle_mod
    rng = np.random.default_rng(11)
    pred = rng.uniform(size=(3, 37, 53)).astype(np.float32)
    tgt = rng.uniform(size=(3, 37, 53)).astype(np.float32)
    loss, grad = R.l1_loss(torch.from_numpy(pred).cuda(), torch.from_numpy(tgt).cuda())
    rl, rg = O.l1_loss_grad(pred, tgt)
    assert abs(float(loss.item()) - rl) <= 1e-6 * rl
    np.testing.assert_allclose(grad.cpu().numpy(), rg, rtol=1e-7)
    # fused Adam with activation epilogues vs the textbook update in FP64
    from paper_2411_19588_amd import optim
    n = 5000
    raw = {"log_scales": rng.normal(-3, 0.5, n), "logits": rng.normal(0, 1, n), "means": rng.normal(0, 1, n)}
    lrs = {"log_scales": 0.005, "logits": 0.05, "means": 1.6e-4}
    acts = {"log_scales": "exp", "logits": "sigmoid", "means": None}
    opt = optim.FusedAdam([optim.Group(name, torch.from_numpy(raw[name].astype(np.float32)).cuda(), lrs[name],
                                       acts[name]) for name in raw])
    ref = {k: (raw[k].astype(np.float32).astype(np.float64), np.zeros(n), np.zeros(n)) for k in raw}
    for step in range(1, 4):
        grads = {k: rng.normal(size=n) for k in raw}
        for grp in opt.groups:
            grp.grad.copy_(torch.from_numpy(grads[grp.name].astype(np.float32)))
        # reference: gradient w.r.t. the activated value chained through the activation
        for k in raw:
            p, m, v = ref[k]
            a = acts[k]
            cur = grp_act = None
            g = grads[k].astype(np.float32).astype(np.float64)
            if a == "exp":
                cur = opt.group(k).activated.double().cpu().numpy()
                g = g * cur
            elif a == "sigmoid":
                cur = opt.group(k).activated.double().cpu().numpy()
                g = g * cur * (1 - cur)
            ref[k] = O.adam_step(p, g, m, v, lrs[k], step)
        opt.step()
        torch.cuda.synchronize()
        for k in raw:
            got = opt.group(k).param.double().cpu().numpy()
            np.testing.assert_allclose(got, ref[k][0], rtol=2e-5, atol=2e-6 * lrs[k] / 1e-3)
    sc, oc = O.activate(opt.group("log_scales").param.cpu().numpy(), opt.group("logits").param.cpu().numpy())
    np.testing.assert_allclose(opt.group("log_scales").activated.cpu().numpy(), sc, rtol=2e-6)
    np.testing.assert_allclose(opt.group("logits").activated.cpu().numpy(), oc, rtol=2e-6)


def test_medium_gradient_deterministic_across_backwards():
    """The medium reduction is deterministic: each view's 16 workgroups sum fixed slices of its
    tiles' partials in a fixed order, and the last one to finish adds the slice sums in slice
    order.  Three backward calls on one forward of a multi-tile, three-view scene give bitwise
    equal medium gradients (the Gaussians' gradients, accumulated by atomics, may differ in the
    last bits), and the counters that pick the last slice start at zero on every call."""
    sc = synth.make_scene(3, n=3000, n_views=3, view_sizes=[(203, 141), (96, 64), (130, 77)])
    rast = U.make_rast(sc)
    rgb, depth, alpha, ctx, d = U.forward(sc, rast)
    g_rgb = torch.from_numpy(np.random.default_rng(3).normal(size=rgb.numel()).astype(np.float32)).cuda()
    meds = []
    for _ in range(3):
        out = rast.backward(ctx, d["means"], d["scales"], d["quats"], d["opacity"], d["sh"], d["medium"], g_rgb)
        torch.cuda.synchronize()
        meds.append(out[5].cpu().numpy().copy())
    assert np.abs(meds[0]).max() > 0.0
    for m in meds[1:]:
        assert np.array_equal(m, meds[0])
    U.say(f"  medium gradient bitwise equal over 3 backwards: {meds[0].reshape(3, 9)[:, :3].tolist()}")
