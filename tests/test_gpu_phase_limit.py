"""Running only the leading depth phases (gs_options.phase_limit): the same images and gradients
as the full schedule when the phases left out would blend nothing, and a truncated render
(GS_STATUS_INCOMPLETE) that gives no gradient and no Adam step when they would not."""
import dataclasses

import numpy as np
import pytest
import torch

from paper_2411_19588_amd import _native as N
from paper_2411_19588_amd import rasterizer as R
from paper_2411_19588_amd import synth
from paper_2411_19588_amd.trainer import TrainStep
from tests import gpu_util as U

pytestmark = pytest.mark.gpu


def _render(sc, **cfg):
    rast = U.make_rast(sc, **cfg)
    rgb, depth, alpha, ctx, d = U.forward(sc, rast)
    return rast, rgb, depth, alpha, ctx, d


def _grads(sc, rast, ctx, d, seed=3):
    g = torch.Generator(device="cuda").manual_seed(seed)
    up = torch.randn(3 * rast.total_pixels, device="cuda", generator=g)
    out = rast.backward(ctx, d["means"], d["scales"], d["quats"], d["opacity"], d["sh"], d["medium"], up)
    torch.cuda.synchronize()
    return [t.clone() for t in out]


@pytest.mark.parametrize("views", [1, 2])
def test_limit_to_the_phases_needed_is_exact(views):
    """1M Gaussians of the 1080p training scene at 480x270 with a 3-phase schedule (nearest 1/128,
    1/32, rest), as one view or as two views of the same pose with different media: the tiles
    terminate early, so fewer phases are needed; a render limited to them reports no truncation,
    equals the full render bit for bit, and so does its gradient up to the order of the float
    atomics."""
    sc = synth.make_scene(2, width=480, height=270, with_target=False)
    if views == 2:
        med = np.stack([sc.medium[0], sc.medium[0][::-1].copy()]).astype(np.float32)
        sc = dataclasses.replace(sc, cameras=[sc.cameras[0], sc.cameras[0]], medium=med)
    cfg = dict(phases=3, phase0_shift=7, phase_growth=2, max_pairs=1 << 24)
    U.say(f"phase limit: full render, {views} view(s)")
    rast, rgb, depth, alpha, ctx, d = _render(sc, **cfg)
    st, _ = rast.read_status(ctx.saved)
    assert st == 0
    k = rast.phases_needed(ctx.saved, ctx.n, ctx.max_pairs)
    U.say(f"phases needed: {k}")
    assert 1 <= k < 3
    ref = _grads(sc, rast, ctx, d)
    rast_k, rgb_k, depth_k, alpha_k, ctx_k, _ = _render(sc, phase_limit=k, **cfg)
    st_k, _ = rast_k.read_status(ctx_k.saved)
    assert st_k == 0
    assert torch.equal(rgb_k, rgb) and torch.equal(depth_k, depth) and torch.equal(alpha_k, alpha)
    got = _grads(sc, rast_k, ctx_k, d)
    # the medium reduction is deterministic; the Gaussians' 2D gradients are float atomics whose
    # order varies between runs, which the projection adjoint amplifies in the quaternions
    for name, a, b in zip(("means", "scales", "quats", "opacity", "sh", "medium"), got, ref):
        if name == "medium":
            assert torch.equal(a, b)
            continue
        a64, b64 = a.double().cpu().numpy(), b.double().cpu().numpy()
        tol = 2e-3 if name == "quats" else 1e-4
        assert np.linalg.norm(a64 - b64) <= tol * np.linalg.norm(b64) + 1e-30, name


def test_cut_short_render_is_flagged_and_gives_no_gradient():
    """A sparse scene (1000 Gaussians, 128x128) whose tiles stay unterminated after the nearest half:
    with phase_limit = 1 of a 2-phase schedule the forward reports GS_STATUS_INCOMPLETE, the adjoint
    writes zero gradients, and the autograd wrapper (which checks the status) renders again with
    every phase."""
    sc = synth.make_scene(0, with_target=False)
    cfg = dict(phases=2, phase0_shift=1)
    rast_full, rgb, depth, alpha, ctx, d = _render(sc, **cfg)
    assert rast_full.phases_needed(ctx.saved, ctx.n, ctx.max_pairs) == 2
    U.say("phase limit: cut-short render")
    rast = U.make_rast(sc, phase_limit=1, **cfg)
    rgb1, depth1, alpha1, ctx1 = rast.forward(d["means"], d["scales"], d["quats"], d["opacity"], d["sh"],
                                              sc.sh_degree, d["medium"], check=False)
    torch.cuda.synchronize()
    st, _ = rast.read_status(ctx1.saved)
    assert st & N.GS_STATUS_INCOMPLETE and not st & N.GS_STATUS_PAIR_OVERFLOW
    assert rast.phases_needed(ctx1.saved, ctx1.n, ctx1.max_pairs) == 2
    for name, g in zip(("means", "scales", "quats", "opacity", "sh", "medium"), _grads(sc, rast, ctx1, d)):
        assert torch.count_nonzero(g).item() == 0, name
    rgb2, depth2, alpha2, ctx2 = rast.forward(d["means"], d["scales"], d["quats"], d["opacity"], d["sh"],
                                              sc.sh_degree, d["medium"])
    torch.cuda.synchronize()
    assert rast.read_status(ctx2.saved)[0] == 0
    assert torch.equal(rgb2, rgb) and torch.equal(depth2, depth) and torch.equal(alpha2, alpha)


def _train(sc, **cfg):
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a))
    tgt = torch.cat([t(x).reshape(-1) for x in sc.targets])
    return TrainStep(t(sc.means), t(sc.log_scales), t(sc.quats), t(sc.logits), t(sc.sh), t(sc.medium),
                     sc.sh_degree, sc.cameras, tgt, R.RasterConfig(**cfg), fused=True)


def test_training_step_with_a_fitted_limit():
    """fit_phase_limit() on the sparse scene keeps every phase (its render needs them); a limit of 1
    makes the fused step a no-op that sets the sticky flag (parameters, moments and the step counter
    unchanged, eagerly and from a replayed graph); with the fitted limit again and the flag cleared,
    steps apply."""
    sc = synth.make_scene(0)
    ts = _train(sc, phases=2, phase0_shift=1)
    ts.size_capacity()
    assert ts.fit_phase_limit() == 2
    stream = torch.cuda.Stream()
    U.say("phase limit: training step")
    with torch.cuda.stream(stream):
        ts.enqueue(stream)
        torch.cuda.synchronize()
        assert ts.skipped() == 0 and int(ts.step_counter.item()) == 1
        before = [(g.param.clone(), g.m.clone(), g.v.clone()) for g in ts.groups]
        ts.set_phase_limit(1)
        ts.enqueue(stream)
        torch.cuda.synchronize()
        assert ts.status(stream)[0] & N.GS_STATUS_INCOMPLETE
        assert ts.skipped() & N.GS_STATUS_INCOMPLETE and int(ts.step_counter.item()) == 1
        ts.capture(stream)
        for _ in range(2):
            ts.replay(stream)
        torch.cuda.synchronize()
        for g, (p, m, v) in zip(ts.groups, before):
            assert torch.equal(g.param, p) and torch.equal(g.m, m) and torch.equal(g.v, v), g.name
        assert int(ts.step_counter.item()) == 1
        ts.set_phase_limit(2)
        ts.clear_skip()
        ts.enqueue(stream)
        torch.cuda.synchronize()
        assert ts.status(stream)[0] == 0 and ts.skipped() == 0 and int(ts.step_counter.item()) == 2
