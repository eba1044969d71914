"""GPU parity of the forward path: keys bit-exact, images within 1e-4 of the FP64 oracle."""
import dataclasses

import numpy as np
import pytest
import torch

from paper_2411_19588_amd import synth
from paper_2411_19588_amd import _native as N
from tests import gpu_util as U

pytestmark = pytest.mark.gpu


def _keys_match(scene, rast, O, opts=None):
    """Full binning (one phase): the stored list equals the oracle's sorted key list bit for bit."""
    assert rast.config.phases == 1
    rgb, depth, alpha, ctx, _ = U.forward(scene, rast)
    k, v, ranges = rast.export_keys(ctx)
    k = k.cpu().numpy().view(np.uint64)
    v = v.cpu().numpy().view(np.uint32)
    ranges = ranges[0].cpu().numpy().astype(np.int64)
    ok, ov, counts = O.keys(scene, opts=opts or O.Options(tile_w=rast.config.tile, tile_h=rast.config.tile))
    assert k.size == ok.size, (k.size, ok.size)
    np.testing.assert_array_equal(k, ok)
    np.testing.assert_array_equal(v, ov)
    np.testing.assert_array_equal(ranges[:, 1] - ranges[:, 0], counts)
    starts = np.concatenate([[0], np.cumsum(counts)[:-1]])
    nz = counts > 0
    np.testing.assert_array_equal(ranges[nz, 0], starts[nz])
    return k.size


def test_keys_bitexact_config0(oracle_mod):
    sc = synth.make_scene(0)
    U.say("keys config0")
    K = _keys_match(sc, U.make_rast(sc, phases=1, tile_cull=False), oracle_mod)
    assert K > 1000


@pytest.mark.parametrize("tile", [16, 8])
def test_keys_bitexact_config1_small(oracle_mod, tile):
    sc = synth.make_scene(1, n=20000, width=203, height=141)
    U.say(f"keys config1 small tile {tile}")
    K = _keys_match(sc, U.make_rast(sc, tile=tile, lds_batch=64 if tile == 8 else 256, phases=1, tile_cull=False),
                    oracle_mod)
    assert K > 20000


@pytest.mark.parametrize("capacity", [6_000_000, 9_000_000])
def test_keys_bitexact_many_sort_tiles(oracle_mod, capacity):
    """5.7e6 pairs at 1600x1067: the tile sort spans ~2800 radix tiles of 2048 keys, several per sort
    workgroup, and its second digit pass covers 5 bits.  A capacity of 9e6 pairs (above the
    8,388,608-key threshold) sorts in radix tiles of 4096 keys instead, two per workgroup."""
    sc = synth.make_scene(1, n=120000)
    U.say(f"keys many sort tiles, capacity {capacity}")
    K = _keys_match(sc, U.make_rast(sc, phases=1, tile_cull=False, max_pairs=capacity), oracle_mod)
    assert K > 5_000_000


def test_keys_bitexact_nine_bit_digit(oracle_mod):
    """400x300 has 475 tiles: tile ids (with the culled id) need 9 bits, sorted in one pass of 512
    digit counters."""
    sc = synth.make_scene(1, n=20000, width=400, height=300)
    U.say("keys nine-bit digit")
    rast = U.make_rast(sc, phases=1, tile_cull=False)
    assert rast.tile_count() == 475
    _keys_match(sc, rast, oracle_mod)


def test_keys_bitexact_seventeen_bit_tile_ids(oracle_mod):
    """Nine 1920x1080 views: 73440 tiles, 17-bit tile ids sorted in two passes (9 + 8 bits)."""
    sc = synth.make_scene(3, n=20000, n_views=9, view_sizes=[(1920, 1080)] * 9)
    U.say("keys seventeen-bit tile ids")
    rast = U.make_rast(sc, phases=1, tile_cull=False, max_pairs=8_000_000)
    assert rast.tile_count() == 9 * 8160
    _keys_match(sc, rast, oracle_mod)


def test_keys_bitexact_multiview(oracle_mod):
    sc = synth.make_scene(3, n=5000, n_views=3, view_sizes=[(96, 64), (130, 77), (64, 64)])
    U.say("keys multiview")
    _keys_match(sc, U.make_rast(sc, phases=1, tile_cull=False), oracle_mod)


def _large_splat_scene():
    """6000 Gaussians at 203x141, three times the usual scale and fainter: about 200 entries whose
    rectangles exceed 32 tiles fall behind the nearest 1/64, into a later depth phase."""
    sc = synth.make_scene(1, n=6000, width=203, height=141)
    ls = (sc.log_scales + np.float32(np.log(3.0))).astype(np.float32)
    lg = (sc.logits - 2.0).astype(np.float32)
    return synth.Scene(**{**sc.__dict__, "log_scales": ls, "scales": np.exp(ls).astype(np.float32), "logits": lg,
                          "opacity": (1.0 / (1.0 + np.exp(-lg))).astype(np.float32)})


@pytest.mark.parametrize("phases,shift,views", [(2, 0, 1), (3, 0, 1), (4, 0, 1), (2, 8, 1), (3, 2, 1),
                                                (2, 6, 3), (3, 3, 3), (2, 6, "large"), (3, 4, "large"),
                                                (8, 14, 1), (6, 10, 3), (2, 7, "huge"), (4, 7, "huge")])
def test_phased_lists_are_exact_prefixes(oracle_mod, phases, shift, views):
    """Depth-progressive binning stores, per tile, a prefix of the oracle's sorted list (bit-exact keys,
    cut at a phase boundary), and the images equal those of full binning bit for bit.  Later phases
    with few front Gaussians leave tiles partially alive, so rows are walked over their alive span;
    the ragged three-view scene puts those rows at several view offsets; the large-splat scene sends
    rectangles of more than 32 tiles to later phases, and the full-resolution scene rectangles of
    more than 256 tiles, which one wave each counts and emits."""
    O = oracle_mod
    if views == 1:
        sc = synth.make_scene(1, n=20000, width=203, height=141)
    elif views == 3:
        sc = synth.make_scene(3, n=20000, n_views=3, view_sizes=[(203, 141), (130, 77), (96, 160)])
    elif views == "huge":
        sc = synth.make_scene(1, n=20000)   # 1600x1067: ~370 rectangles of more than 256 tiles past phase 0
    else:
        sc = _large_splat_scene()
    U.say(f"phased prefixes {phases} shift {shift} views {views}")
    rast = U.make_rast(sc, phases=phases, phase0_shift=shift, tile_cull=False)
    rgb, depth, alpha, ctx, _ = U.forward(sc, rast)
    k, v, ranges = rast.export_keys(ctx)
    k = k.cpu().numpy().view(np.uint64)
    v = v.cpu().numpy().view(np.uint32)
    ranges = ranges.cpu().numpy().astype(np.int64)
    ok, ov, counts = O.keys(sc)
    starts = np.concatenate([[0], np.cumsum(counts)[:-1]])
    stored = 0
    for t in range(counts.size):
        parts = [(ranges[p, t, 0], ranges[p, t, 1]) for p in range(phases) if ranges[p, t, 1] > ranges[p, t, 0]]
        gk = np.concatenate([k[a:b] for a, b in parts]) if parts else np.zeros(0, np.uint64)
        gv = np.concatenate([v[a:b] for a, b in parts]) if parts else np.zeros(0, np.uint32)
        n_t = gk.size
        assert n_t <= counts[t]
        np.testing.assert_array_equal(gk, ok[starts[t]: starts[t] + n_t])
        np.testing.assert_array_equal(gv, ov[starts[t]: starts[t] + n_t])
        stored += n_t
    assert stored == k.size
    full = U.forward(sc, U.make_rast(sc, phases=1))[:3]
    for a, b in zip((rgb, depth, alpha), full):
        assert torch.equal(a, b)


@pytest.mark.parametrize("phases,shift,scene", [(2, 6, "large"), (3, 4, "large"), (2, 7, "huge"), (4, 7, "huge")])
def test_large_rectangles_in_later_phases_with_culling(phases, shift, scene):
    """Rectangles of more than 32 (and, at 1600x1067, more than 256) tiles in later phases, with the
    exact tile culling on: images equal those of full binning without culling bit for bit."""
    sc = _large_splat_scene() if scene == "large" else synth.make_scene(1, n=20000)
    U.say(f"large rectangles, culling, phases {phases} shift {shift}")
    got = U.forward(sc, U.make_rast(sc, phases=phases, phase0_shift=shift, tile_cull=True))
    ref = U.forward(sc, U.make_rast(sc, phases=1, tile_cull=False))
    for a, b in zip(got[:3], ref[:3]):
        assert torch.equal(a, b)


def _tile_max_alpha(O, scene, cam, tiles, gauss, tile_w):
    """FP64 maximum over the pixel centres of each tile of alpha = o exp(-q/2) of the paired Gaussian."""
    pr = O.project(scene, cam)
    tx_n = -(-cam.width // tile_w)
    out = np.zeros(tiles.size)
    off = np.arange(tile_w) + 0.5
    for s0 in range(0, tiles.size, 4096):
        t = tiles[s0:s0 + 4096]
        g = gauss[s0:s0 + 4096]
        px = (t % tx_n)[:, None] * tile_w + off[None, :]          # (m, tile_w) pixel-centre columns
        py = (t // tx_n)[:, None] * tile_w + off[None, :]
        vx = px < cam.width
        vy = py < cam.height
        dx = px - pr["mean2d"][g, 0][:, None]
        dy = py - pr["mean2d"][g, 1][:, None]
        a, b, c = (pr["conic"][g, i][:, None, None] for i in range(3))
        q = a * dx[:, None, :] ** 2 + 2 * b * dx[:, None, :] * dy[:, :, None] + c * dy[:, :, None] ** 2
        al = scene.opacity[g].astype(np.float64)[:, None, None] * np.exp(-0.5 * q)
        al = np.where(vy[:, :, None] & vx[:, None, :], al, 0.0)
        out[s0:s0 + 4096] = al.reshape(al.shape[0], -1).max(axis=1)
    return out


@pytest.mark.parametrize("tile", [16, 8])
def test_tile_cull_drops_only_non_contributing_pairs(oracle_mod, tile):
    """With exact tile culling each tile keeps a subsequence of the oracle's (rectangle) list; every
    dropped pair has alpha < alpha_min at all of the tile's pixel centres (FP64), few kept pairs
    could have been dropped, and the images equal those without culling bit for bit."""
    O = oracle_mod
    sc = synth.make_scene(1, n=20000, width=203, height=141)
    cam = sc.cameras[0]
    U.say(f"tile cull tile {tile}")
    lb = 64 if tile == 8 else 256
    rast = U.make_rast(sc, tile=tile, lds_batch=lb, phases=1, tile_cull=True)
    rgb, depth, alpha, ctx, _ = U.forward(sc, rast)
    k, v, ranges = rast.export_keys(ctx)
    k = k.cpu().numpy().view(np.uint64)
    v = v.cpu().numpy().view(np.uint32).astype(np.int64)
    ranges = ranges[0].cpu().numpy().astype(np.int64)
    ok, ov, counts = O.keys(sc, opts=O.Options(tile_w=tile, tile_h=tile))
    starts = np.concatenate([[0], np.cumsum(counts)[:-1]])
    dropped_t, dropped_g, kept_t, kept_g = [], [], [], []
    for t in np.nonzero(counts)[0]:
        full_k = ok[starts[t]: starts[t] + counts[t]]
        full_v = ov[starts[t]: starts[t] + counts[t]].astype(np.int64)
        a, b = ranges[t]
        gk, gv = k[a:b], v[a:b]
        # subsequence in the same order: keys are unique per (tile, depth, index) after the value
        mask = np.isin(full_v, gv)
        np.testing.assert_array_equal(full_v[mask], gv)
        np.testing.assert_array_equal(full_k[mask], gk)
        dropped_t.append(np.full(int((~mask).sum()), t))
        dropped_g.append(full_v[~mask])
        kept_t.append(np.full(gv.size, t))
        kept_g.append(gv)
    dt, dg = np.concatenate(dropped_t), np.concatenate(dropped_g)
    kt, kg = np.concatenate(kept_t), np.concatenate(kept_g)
    assert dt.size > 0.1 * ok.size, "culling should drop a sizeable share of the rectangle pairs"
    amin = 1.0 / 255.0
    dmax = _tile_max_alpha(O, sc, cam, dt, dg, tile)
    assert np.all(dmax < amin), (dmax.max(), amin)
    kmax = _tile_max_alpha(O, sc, cam, kt, kg, tile)
    loose = int(np.sum(kmax < amin))
    U.say(f"  rectangle pairs {ok.size}, kept {kt.size}, dropped {dt.size}, kept but below alpha_min {loose}")
    assert loose <= 0.01 * kt.size
    for phases in (1, 3):
        ref = U.forward(sc, U.make_rast(sc, tile=tile, lds_batch=lb, phases=phases, tile_cull=False))[:3]
        got = U.forward(sc, U.make_rast(sc, tile=tile, lds_batch=lb, phases=phases, tile_cull=True))[:3]
        for x, y in zip(got, ref):
            assert torch.equal(x, y)


def _image_match(scene, rast, O, opts=None, v=0):
    rgb, depth, alpha, ctx, _ = U.forward(scene, rast)
    st, _ = rast.read_status(ctx.saved)
    assert st == 0
    cam = scene.cameras[v]
    pix = U.pixel_list(cam.width, cam.height)
    orc = O.render(scene, cam, scene.medium[v], opts or O.Options(depth_mode=rast.config.depth_mode),
                   pixels=pix, variants=4)
    g = U.gather_view(rgb, depth, alpha, rast, v, pix)
    return U.compare_pixels(*g, orc)


def test_image_config0(oracle_mod):
    sc = synth.make_scene(0)
    U.say("image config0")
    n_main, n_var, worst = _image_match(sc, U.make_rast(sc), oracle_mod)
    U.say(f"  main {n_main} variant {n_var} worst {worst:.2e}")


def _edge_opacity_scene():
    """The 1,000-Gaussian scene with opacities of exactly 0, below 0, 1e-30 and 1 mixed in (the
    record stores log2 o and 1/o: an opacity <= 0 stores -inf and 0 and must never blend)."""
    sc = synth.make_scene(0)
    op = sc.opacity.copy()
    op[0::7] = 0.0
    op[1::7] = -0.25
    op[2::7] = 1e-30
    op[3::7] = 1.0
    return dataclasses.replace(sc, opacity=op)


def test_image_opacity_edge_values(oracle_mod):
    sc = _edge_opacity_scene()
    U.say("image with edge opacities")
    n_main, n_var, worst = _image_match(sc, U.make_rast(sc), oracle_mod)
    U.say(f"  main {n_main} variant {n_var} worst {worst:.2e}")


def test_image_config1_small(oracle_mod):
    sc = synth.make_scene(1, n=20000, width=203, height=141)
    U.say("image config1 small")
    n_main, n_var, worst = _image_match(sc, U.make_rast(sc), oracle_mod)
    U.say(f"  main {n_main} variant {n_var} worst {worst:.2e}")


def test_image_logistic_depth(oracle_mod):
    sc = synth.make_scene(1, n=8000, width=100, height=70)
    U.say("image logistic depth")
    _image_match(sc, U.make_rast(sc, depth_mode=1), oracle_mod, oracle_mod.Options(depth_mode=1))


def test_image_multiview(oracle_mod):
    sc = synth.make_scene(3, n=5000, n_views=3, view_sizes=[(96, 64), (130, 77), (64, 64)])
    rast = U.make_rast(sc)
    U.say("image multiview")
    for v in range(3):
        _image_match(sc, rast, oracle_mod, v=v)


def test_image_max_views(oracle_mod):
    """GS_MAX_VIEWS views of uneven small sizes in one pipeline (the largest view table): every
    view's image against the oracle, in the automatic several-view schedule."""
    V = N.GS_MAX_VIEWS
    sizes = [(16 + 8 * (v % 3), 16 + 8 * (v % 2)) for v in range(V)]
    sc = synth.make_scene(3, n=600, n_views=V, view_sizes=sizes)
    rast = U.make_rast(sc)
    U.say(f"image {V} views")
    for v in range(V):
        _image_match(sc, rast, oracle_mod, v=v)


@pytest.mark.parametrize("cfg", [dict(lds_batch=256), dict(lds_batch=128), dict(persistent=True),
                                 dict(pixels_per_lane=1), dict(pixels_per_lane=4, lds_batch=64),
                                 dict(pixels_per_lane=1, persistent=True, lds_batch=128),
                                 dict(pixels_per_lane=4, persistent=True),
                                 dict(record_fetch="scalar", pixels_per_lane=1),
                                 dict(record_fetch="scalar", pixels_per_lane=2),
                                 dict(record_fetch="scalar", pixels_per_lane=4, persistent=True),
                                 dict(record_fetch="scalar", pixels_per_lane=1, persistent=True),
                                 dict(tile=8, lds_batch=64), dict(tile=8, lds_batch=64, persistent=True),
                                 dict(tile=8, lds_batch=64, record_fetch="scalar"), dict(persistent=2),
                                 dict(persistent=2, pixels_per_lane=4, record_fetch="scalar", phases=3, phase0_shift=6),
                                 dict(persistent=2, tile=8, lds_batch=64)])
def test_launch_variants_bitwise_equal(cfg):
    """Every tile shape / split / batch / record fetch / persistent variant walks each pixel's
    Gaussians in the same order with the same operations, so the images are bitwise identical."""
    sc = synth.make_scene(1, n=20000, width=203, height=141)
    U.say(f"variant {cfg}")
    base = U.forward(sc, U.make_rast(sc))[:3]
    other = U.forward(sc, U.make_rast(sc, **cfg))[:3]
    for a, b in zip(base, other):
        assert torch.equal(a, b)


def test_empty_scene_and_all_culled(oracle_mod):
    sc = synth.make_scene(0, n=50, width=40, height=24)
    rast = U.make_rast(sc)
    med = torch.from_numpy(sc.medium).cuda()
    z = torch.zeros((3, 0), device="cuda")
    rgb, depth, alpha, ctx = rast.forward(z, z, torch.zeros((4, 0), device="cuda"), torch.zeros(0, device="cuda"),
                                          torch.zeros((3, 0), device="cuda"), 0, med)
    torch.cuda.synchronize()
    binf = sc.medium[0, 6:9]
    expect = np.where(sc.medium[0, 3:6] > 0, binf, 0.0).astype(np.float32)
    r = rgb.view(3, -1).cpu().numpy()
    np.testing.assert_array_equal(r, np.repeat(expect[:, None], r.shape[1], axis=1))
    assert torch.count_nonzero(alpha) == 0 and torch.count_nonzero(depth) == 0
    # all Gaussians behind the camera
    means = sc.means.copy()
    means[2] = -means[2]
    sc2 = synth.Scene(**{**sc.__dict__, "means": means})
    rgb2, _, alpha2, ctx2, _ = U.forward(sc2, rast)
    assert torch.count_nonzero(alpha2) == 0
    np.testing.assert_array_equal(rgb2.view(3, -1).cpu().numpy(), r)


@pytest.mark.parametrize("phases", [1, 3])
def test_pair_overflow_reported_and_recovered(oracle_mod, phases):
    sc = synth.make_scene(0)
    rast = U.make_rast(sc, max_pairs=100, phases=phases)
    d = U.to_dev(sc)
    _, _, _, ctx = rast.forward(d["means"], d["scales"], d["quats"], d["opacity"], d["sh"], 0, d["medium"],
                                check=False)
    st, need = rast.read_status(ctx.saved)
    ok, _, _ = oracle_mod.keys(sc)
    assert st & N.GS_STATUS_PAIR_OVERFLOW
    assert need == ok.size if phases == 1 else 100 < need <= ok.size
    # the checked path grows the capacity and renders correctly
    rgb, depth, alpha, ctx = rast.forward(d["means"], d["scales"], d["quats"], d["opacity"], d["sh"], 0,
                                          d["medium"])
    assert phases > 1 or ctx.max_pairs >= ok.size
    ref = U.forward(sc, U.make_rast(sc))[:3]
    assert torch.equal(rgb, ref[0])


def test_pair_overflow_in_a_later_phase():
    """A capacity that holds exactly phase 0's stored pairs overflows in a later phase (whose pairs
    the balanced later-phase emission writes): the status reports it, the needed count exceeds the
    capacity, and the checked path grows the capacity and renders the reference images."""
    sc = synth.make_scene(3, n=2000, n_views=3, view_sizes=[(64, 48), (80, 40), (48, 48)])
    d = U.to_dev(sc)
    args = (d["means"], d["scales"], d["quats"], d["opacity"], d["sh"], sc.sh_degree, d["medium"])
    U.say("pair overflow in a later phase")
    rast = U.make_rast(sc, max_pairs=1, phases=3, phase0_shift=6)
    _, _, _, ctx = rast.forward(*args, check=False)
    st, need0 = rast.read_status(ctx.saved)
    assert st & N.GS_STATUS_PAIR_OVERFLOW and need0 > 1   # phase 0's stored pairs
    rast = U.make_rast(sc, max_pairs=need0, phases=3, phase0_shift=6)
    _, _, _, ctx = rast.forward(*args, check=False)
    st, need = rast.read_status(ctx.saved)
    assert st & N.GS_STATUS_PAIR_OVERFLOW and need > need0
    rgb, depth, alpha, ctx = rast.forward(*args)
    assert ctx.max_pairs >= need
    ref = U.forward(sc, U.make_rast(sc, phases=3, phase0_shift=6))[:3]
    assert torch.equal(rgb, ref[0]) and torch.equal(depth, ref[1]) and torch.equal(alpha, ref[2])


def test_nonfinite_input_flagged_and_culled(oracle_mod):
    sc = synth.make_scene(0, n=300, width=64, height=64)
    bad = synth.Scene(**{**sc.__dict__, "means": sc.means.copy()})
    bad.means[0, 5] = np.nan
    rast = U.make_rast(bad)
    rgb, depth, alpha, ctx, _ = U.forward(bad, rast)
    st, _ = rast.read_status(ctx.saved)
    assert st & N.GS_STATUS_NONFINITE_INPUT
    keep = np.arange(sc.n) != 5
    ref_scene = synth.Scene(means=sc.means[:, keep], log_scales=sc.log_scales[:, keep], scales=sc.scales[:, keep],
                            quats=sc.quats[:, keep], logits=sc.logits[keep], opacity=sc.opacity[keep],
                            sh=sc.sh[:, keep], sh_degree=0, cameras=sc.cameras, medium=sc.medium)
    ref = U.forward(ref_scene, U.make_rast(ref_scene))[:3]
    assert torch.equal(rgb, ref[0])


def test_longest_first_queue_several_views_bitwise_equal():
    """The longest-first persistent queue (tiles of every view sorted by list length before each
    phase's pass) renders the same images as one workgroup per tile, over views of uneven size."""
    sizes = [(203, 141), (97, 61), (160, 120)]
    sc = synth.make_scene(3, n=8000, n_views=3, view_sizes=sizes)
    U.say("longest-first queue, 3 views")
    base = U.forward(sc, U.make_rast(sc, phases=3, phase0_shift=5))[:3]
    other = U.forward(sc, U.make_rast(sc, phases=3, phase0_shift=5, persistent=2))[:3]
    for a, b in zip(base, other):
        assert torch.equal(a, b)
