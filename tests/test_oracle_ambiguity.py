"""Pins for the oracle's near-threshold variants (the "several results correct" rule).

Where FP32 and FP64 may legitimately take different discrete decisions -- the
alpha skip (alpha vs 1/255) and the termination (T (1 - alpha) vs 1e-4) -- the
oracle flags every decision whose relative margin is within `band` and renders
the pixel again with each flagged decision flipped.  The GPU image is accepted
against any of these variants, and the gradient tests mask flagged pixels, so a
bug here (the wrong decision flipped, a variant written into the wrong slot, a
flag on an unambiguous pixel) would silently widen what passes.

Each case places Gaussians exactly on a pixel centre, where the exponent is
exactly 0 and alpha equals the opacity, so every decision is known in closed
form: the variants must equal the closed-form composites of the walk with that
Gaussian kept or skipped, or stopped one Gaussian earlier or later.
"""
import math

import numpy as np
import pytest

from tests.test_oracle_pins import _cam, _colour_of, _scene

MED = np.array([0.2, 0.3, 0.4, 0.1, 0.25, 0.45, 0.05, 0.15, 0.28], np.float64)
PIX = np.array([[8, 8]], np.int32)   # the pixel whose centre (8.5, 8.5) is every Gaussian's 2D mean


def _cam_centre():
    return _cam(16, 16, 30.0, cx=8.5, cy=8.5)


def _composite(cols, alphas, ds):
    """Front-to-back composite of the listed contributors (all blended) and the medium epilogue."""
    T, C, D, W = 1.0, np.zeros(3), 0.0, 0.0
    for c, a, d in zip(cols, alphas, ds):
        w = a * T
        C = C + w * c
        D += w * d
        W += w
        T *= 1.0 - a
    Bd, Bb, Binf = MED[:3], MED[3:6], MED[6:]
    if W == 0.0:
        return np.r_[np.where(Bb > 0, Binf, 0.0), 0.0, 0.0]
    z = D / W
    return np.r_[C * np.exp(-Bd * z) + Binf * (1 - np.exp(-Bb * z)), z, W]


def _out(o, k=0):
    return np.r_[o["rgb"][k], o["depth"][k], o["alpha"][k]]


def _f32(x):
    return float(np.float32(x))


def _stack_scene(opacities, depths):
    n = len(opacities)
    cols = [[0.1 + 0.15 * i, 0.8 - 0.1 * i, 0.3 + 0.05 * i] for i in range(n)]
    sc = _scene([[0, 0, d] for d in depths], [[0.02] * 3] * n, [[1, 0, 0, 0]] * n, opacities, colors=cols,
                medium=MED.astype(np.float32))
    return sc, [_colour_of(sc, i) for i in range(n)]


@pytest.mark.parametrize("rel", [+0.3, -0.3])
def test_skip_decision_inside_band_has_the_flipped_variant(oracle_mod, rel):
    O = oracle_mod
    opts = O.Options()
    amin = opts.alpha_min
    o = _f32(amin * (1.0 + rel * opts.band))
    margin = (o - amin) / amin
    assert 0 < abs(margin) <= opts.band and np.sign(margin) == np.sign(rel)   # precondition
    d = 3.0
    sc, cols = _stack_scene([o], [d])
    out = O.render(sc, _cam_centre(), MED, opts, pixels=PIX, variants=4)
    kept = _composite(cols, [o], [d])
    skipped = _composite([], [], [])
    main, var = (kept, skipped) if rel > 0 else (skipped, kept)
    np.testing.assert_allclose(_out(out), main, rtol=1e-12, atol=1e-15)
    assert out["nvar"][0] == 1
    np.testing.assert_allclose(out["var"][0, 0], var, rtol=1e-12, atol=1e-15)


@pytest.mark.parametrize("rel", [+3.0, -3.0])
def test_skip_decision_outside_band_has_no_variant(oracle_mod, rel):
    O = oracle_mod
    opts = O.Options()
    o = _f32(opts.alpha_min * (1.0 + rel * opts.band))
    sc, cols = _stack_scene([o], [3.0])
    out = O.render(sc, _cam_centre(), MED, opts, pixels=PIX, variants=4)
    assert out["nvar"][0] == 0
    ref = _composite(cols, [o], [3.0]) if rel > 0 else _composite([], [], [])
    np.testing.assert_allclose(_out(out), ref, rtol=1e-12, atol=1e-15)


def _termination_stack(opts, rel, front=None):
    """Opacities (front Gaussian optional), 0.95, 0.95, a, 0.5 with T (1 - a) = t_min (1 + rel band)
    before the third of the stack (exactly, up to the FP32 rounding of a)."""
    ops = [] if front is None else [front]
    ops += [_f32(0.95), _f32(0.95)]
    T = np.prod([1.0 - x for x in ops])
    a = _f32(1.0 - opts.t_min * (1.0 + rel * opts.band) / T)
    margin = (T * (1.0 - a) - opts.t_min) / opts.t_min
    assert 0 < abs(margin) <= opts.band and np.sign(margin) == np.sign(rel)   # precondition
    assert a < opts.alpha_max
    ops += [a, _f32(0.5)]
    depths = [1.5 + 0.5 * i for i in range(len(ops))]
    return ops, depths


@pytest.mark.parametrize("rel", [+0.3, -0.3])
def test_termination_inside_band_has_the_walk_stopped_one_later_or_earlier(oracle_mod, rel):
    O = oracle_mod
    opts = O.Options()
    ops, ds = _termination_stack(opts, rel)
    sc, cols = _stack_scene(ops, ds)
    out = O.render(sc, _cam_centre(), MED, opts, pixels=PIX, variants=4)
    three = _composite(cols[:3], ops[:3], ds[:3])   # the fourth (alpha 0.5) always stops the walk
    two = _composite(cols[:2], ops[:2], ds[:2])
    main, var = (three, two) if rel > 0 else (two, three)
    np.testing.assert_allclose(_out(out), main, rtol=1e-12, atol=1e-15)
    assert out["ncontrib"][0] == (3 if rel > 0 else 2)
    assert out["nvar"][0] == 1
    np.testing.assert_allclose(out["var"][0, 0], var, rtol=1e-12, atol=1e-15)


def test_termination_outside_band_has_no_variant(oracle_mod):
    O = oracle_mod
    opts = O.Options()
    # T = 2.5e-4 after the 3rd; the 4th would leave 7.5e-5: both decisions 25 % or more from t_min
    ops = [_f32(0.95), _f32(0.95), _f32(0.9), _f32(0.7)]
    ds = [1.5, 2.0, 2.5, 3.0]
    sc, cols = _stack_scene(ops, ds)
    out = O.render(sc, _cam_centre(), MED, opts, pixels=PIX, variants=4)
    assert out["nvar"][0] == 0
    np.testing.assert_allclose(_out(out), _composite(cols[:3], ops[:3], ds[:3]), rtol=1e-12, atol=1e-15)


def test_two_ambiguous_decisions_give_three_variants_in_mask_order(oracle_mod):
    """A front Gaussian with alpha just above 1/255 and a later termination just above t_min: the
    variants are (front skipped), (stopped one earlier), (both), in that order."""
    O = oracle_mod
    opts = O.Options()
    a0 = _f32(opts.alpha_min * (1.0 + 0.3 * opts.band))
    ops, ds = _termination_stack(opts, +0.3, front=a0)
    sc, cols = _stack_scene(ops, ds)
    out = O.render(sc, _cam_centre(), MED, opts, pixels=PIX, variants=8)
    # main: front, 0.95, 0.95, a (the 0.5 stops the walk)
    np.testing.assert_allclose(_out(out), _composite(cols[:4], ops[:4], ds[:4]), rtol=1e-12, atol=1e-15)
    assert out["nvar"][0] == 3
    # front skipped: T before the third of the stack is larger by 1/(1 - a0), so it blends
    # unambiguously and the 0.5 still stops the walk
    v1 = _composite(cols[1:4], ops[1:4], ds[1:4])
    v2 = _composite(cols[:3], ops[:3], ds[:3])        # stopped before the third of the stack
    v3 = _composite(cols[1:3], ops[1:3], ds[1:3])     # both flipped
    for j, ref in enumerate((v1, v2, v3)):
        np.testing.assert_allclose(out["var"][0, j], ref, rtol=1e-12, atol=1e-15, err_msg=f"variant {j}")
    # fewer variant slots than combinations: the first ones in mask order
    out2 = O.render(sc, _cam_centre(), MED, opts, pixels=PIX, variants=2)
    assert out2["nvar"][0] == 2
    np.testing.assert_allclose(out2["var"][0], out["var"][0, :2], rtol=0, atol=0)


def test_variants_land_in_their_pixels_slots(oracle_mod):
    """Ambiguous, unambiguous and ambiguous pixels in one call: only the ambiguous ones have
    variants, each in its own row."""
    O = oracle_mod
    opts = O.Options()
    o = _f32(opts.alpha_min * (1.0 + 0.3 * opts.band))
    sc, cols = _stack_scene([o], [3.0])
    pix = np.array([[8, 8], [0, 0], [8, 8], [15, 3]], np.int32)
    out = O.render(sc, _cam_centre(), MED, opts, pixels=pix, variants=3)
    np.testing.assert_array_equal(out["nvar"], [1, 0, 1, 0])
    empty = _composite([], [], [])
    np.testing.assert_allclose(out["var"][0, 0], empty, rtol=1e-12, atol=1e-15)
    np.testing.assert_array_equal(out["var"][2], out["var"][0])
    np.testing.assert_array_equal(out["var"][1], 0.0)
    np.testing.assert_array_equal(out["var"][3], 0.0)
    np.testing.assert_allclose(_out(out, 1), empty, rtol=0, atol=0)


def test_band_scales_the_flag(oracle_mod):
    """The same pixel is flagged under a wide band and not under a narrow one."""
    O = oracle_mod
    base = O.Options()
    o = _f32(base.alpha_min * (1.0 + 5e-5))
    sc, _ = _stack_scene([o], [3.0])
    wide = O.render(sc, _cam_centre(), MED, O.Options(band=1e-4), pixels=PIX, variants=2)
    narrow = O.render(sc, _cam_centre(), MED, O.Options(band=1e-5), pixels=PIX, variants=2)
    assert wide["nvar"][0] == 1 and narrow["nvar"][0] == 0
    np.testing.assert_array_equal(_out(wide), _out(narrow))
    assert math.isfinite(wide["var"][0, 0, 0])
