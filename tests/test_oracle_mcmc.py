"""Pins for the MCMC densification oracle: the split rule against numerical quadrature of the
stacked copies' opacity profile and the exact stacked opacity, the draws against an independent
search and their frequencies, relocation and addition invariants, the Langevin noise against a
quaternion-sandwich covariance and its opacity gate, and the regularisers' gradients by central
differences."""
import math

import numpy as np
import pytest

from oracle import mcmc as M

GROUP_SHAPES = dict(means=3, log_scales=3, quats=4, logits=1, sh=12)


def _state(n, cap, seed=0, dead_frac=0.2):
    rng = np.random.default_rng(seed)
    st = {}
    for g, k in GROUP_SHAPES.items():
        shape = (k, cap) if k > 1 else (cap,)
        st[g] = rng.normal(size=shape).astype(np.float32)
        st["m_" + g] = rng.normal(size=shape).astype(np.float32)
        st["v_" + g] = rng.uniform(size=shape).astype(np.float32)
    st["log_scales"] = rng.normal(-3, 0.5, size=(3, cap)).astype(np.float32)
    st["scales"] = np.exp(st["log_scales"].astype(np.float64)).astype(np.float32)
    o = rng.uniform(0.12, 0.99, size=cap)
    dead = rng.uniform(size=cap) < dead_frac
    o[dead] = rng.uniform(0.001, 0.1, size=int(dead.sum()))
    st["opacity"] = o.astype(np.float32)
    st["logits"] = np.log(o / (1 - o)).astype(np.float32)
    return st


@pytest.mark.parametrize("N", [1, 2, 3, 7, 20, 51])
@pytest.mark.parametrize("o", [0.05, 0.3, 0.9, 0.995])
def test_split_keeps_stacked_opacity_and_profile_integral(N, o):
    s = np.array([0.7])
    o_new, s_new = M.split(o, s, N)
    if o_new > M.MIN_OPACITY and o_new < 1 - 2 ** -23:
        # N copies on one ray composite to the original opacity (exactly, away from the clamps)
        assert 1 - (1 - o_new) ** N == pytest.approx(o, rel=1e-12)
    # the stacked copies' opacity profile along an axis integrates to the original's
    x = np.linspace(-12 * max(s[0], s_new[0]), 12 * max(s[0], s_new[0]), 400001)
    g_new = o_new * np.exp(-0.5 * (x / s_new[0]) ** 2)
    stacked = 1 - (1 - g_new) ** N
    orig = o * np.exp(-0.5 * (x / s[0]) ** 2)
    assert np.trapezoid(stacked, x) == pytest.approx(np.trapezoid(orig, x), rel=1e-9)


def test_split_sum_matches_the_single_sum_identity():
    """sum_{m<=N} C(m-1, k) = C(N, k+1) turns the double sum into one sum, evaluated here with 60
    significant digits at the opacities the split produces."""
    import decimal
    ctx = decimal.Context(prec=60)
    for N in (1, 2, 5, 13, 51):
        for o in (0.01, 0.2, 0.7, 0.99, 1 - 2 ** -23):
            a = 1.0 - (1.0 - o) ** (1.0 / N)
            A = decimal.Decimal(a)
            single = sum(ctx.multiply(ctx.multiply((-1) ** (j - 1) * math.comb(N, j), ctx.power(A, j)),
                                      ctx.divide(1, ctx.sqrt(decimal.Decimal(j)))) for j in range(1, N + 1))
            assert M.split_sum(N, a) == pytest.approx(float(single), rel=1e-9)


def test_draws_follow_the_integer_intervals_and_the_weights():
    rng = np.random.default_rng(1)
    w = rng.integers(0, 1 << 24, size=50)
    w[[3, 17, 40]] = 0
    r = rng.integers(0, 1 << 32, size=20000, dtype=np.uint64)
    src = M.draw(w, r)
    P = int(w.sum())
    starts = np.concatenate([[0], np.cumsum(w)])
    for j in range(0, 20000, 997):   # brute force: the interval holding t
        t = (int(r[j]) * P) >> 32
        i = [k for k in range(50) if starts[k] <= t < starts[k] + w[k]]
        assert i == [src[j]]
    assert not np.isin(src, [3, 17, 40]).any()
    freq = np.bincount(src, minlength=50) / len(src)
    assert np.allclose(freq, w / P, atol=0.01)


def test_weights_are_exact_floor_and_skip_dead():
    o = np.array([0.1, 0.1000001, 0.5, 1e-7, 0.999], np.float32)
    w = M.weights(o, 5, dead_opacity=0.1)
    assert w[0] == 0 and w[3] == 0
    assert w[1] == math.floor(float(o[1]) * 2 ** 24) and w[2] == 1 << 23
    assert np.array_equal(M.weights(o, 5, live_only=False), np.floor(o.astype(np.float64) * 2 ** 24).astype(np.int64))


def test_relocation_moves_dead_onto_live_and_resets_moments():
    n = cap = 400
    st = _state(n, cap, seed=2)
    r = np.random.default_rng(3).integers(0, 1 << 32, size=n, dtype=np.uint64)
    new, dead, src = M.relocate(st, n, r)
    assert len(dead) > 20 and len(src) == len(dead)
    assert np.all(st["opacity"][src] > 0.1)                     # sources are live
    counts = np.bincount(src, minlength=cap)
    for j, (d, s) in enumerate(zip(dead, src)):
        for g in M.GROUPS + ("scales", "opacity"):
            assert np.array_equal(new[g][..., d], new[g][..., s])
        o_new, s_new = M.split(st["opacity"][s], st["scales"][:, s], counts[s] + 1)
        assert new["opacity"][s] == np.float32(o_new)
        np.testing.assert_allclose(new["scales"][:, s], s_new, rtol=1e-6)
        np.testing.assert_allclose(1 / (1 + np.exp(-new["logits"][s].astype(np.float64))), o_new, rtol=1e-6)
    touched = np.union1d(dead, src)
    untouched = np.setdiff1d(np.arange(cap), touched)
    for g in M.GROUPS:
        assert np.all(new["m_" + g][..., touched] == 0) and np.all(new["v_" + g][..., touched] == 0)
        assert np.array_equal(new["m_" + g][..., untouched], st["m_" + g][..., untouched])
        assert np.array_equal(new[g][..., untouched], st[g][..., untouched])
    # each source and its copies carry the original's stacked opacity
    for s in np.unique(src):
        Nc = counts[s] + 1
        assert 1 - (1 - float(new["opacity"][s])) ** Nc == pytest.approx(float(st["opacity"][s]), rel=1e-5)


def test_addition_appends_copies_up_to_capacity():
    n, cap = 300, 310
    st = _state(cap, cap, seed=4)
    assert M.add_count(n, cap) == 10 and M.add_count(100, 1000) == 5 and M.add_count(cap, cap) == 0
    r = np.random.default_rng(5).integers(0, 1 << 32, size=cap, dtype=np.uint64)
    new, n2, src = M.add(st, n, cap, r)
    assert n2 == cap and len(src) == 10 and np.all(src < n)
    for j, s in enumerate(src):
        for g in M.GROUPS + ("scales", "opacity"):
            assert np.array_equal(new[g][..., n + j], new[g][..., s])
        for g in M.GROUPS:
            assert np.all(new["m_" + g][..., n + j] == 0)


def test_noise_uses_the_covariance_and_its_opacity_gate():
    rng = np.random.default_rng(6)
    n = 5
    means = rng.normal(size=(3, n))
    scales = rng.uniform(0.05, 0.5, size=(3, n))
    quats = rng.normal(size=(4, n))
    eta = rng.normal(size=(3, n))
    opacity = np.array([0.001, 0.002, 0.5, 0.9, 0.9999])
    out = M.noise(means, scales, quats, opacity, eta, 1.6e-4, n)
    for i in range(n):
        q = quats[:, i] / np.linalg.norm(quats[:, i])
        # covariance by rotating the axis-aligned one with the quaternion sandwich q v q*
        def rot(v):
            w, x, y, z = q
            u = np.array([x, y, z])
            return v + 2 * np.cross(u, np.cross(u, v) + w * v)
        Rm = np.stack([rot(e) for e in np.eye(3)], 1)
        S = Rm @ np.diag(scales[:, i] ** 2) @ Rm.T
        gate = 1 / (1 + np.exp(-100 * ((1 - opacity[i]) - 0.995)))
        np.testing.assert_allclose(out[:, i] - means[:, i], 1.6e-4 * 5e5 * gate * S @ eta[:, i], rtol=1e-10,
                                   atol=1e-15)
    # opaque Gaussians barely move, nearly transparent ones take the full step
    assert np.abs(out[:, 4] - means[:, 4]).max() < 1e-20 + 1e-6 * np.abs(out[:, 0] - means[:, 0]).max()


def test_regulariser_gradients_by_central_differences():
    rng = np.random.default_rng(7)
    n = 40
    o = rng.uniform(0.1, 0.9, size=n)
    s = rng.uniform(0.01, 0.3, size=(3, n))
    L = lambda o_, s_: M.REG_OPACITY * np.abs(o_).mean() + M.REG_SCALE * np.abs(s_).mean()
    go, gs = M.reg_grads(n)
    h = 1e-6
    for i in (0, 7, 39):
        op, om = o.copy(), o.copy()
        op[i] += h
        om[i] -= h
        assert go == pytest.approx((L(op, s) - L(om, s)) / (2 * h), rel=1e-6)
        sp, sm = s.copy(), s.copy()
        sp[1, i] += h
        sm[1, i] -= h
        assert gs == pytest.approx((L(o, sp) - L(o, sm)) / (2 * h), rel=1e-6)
