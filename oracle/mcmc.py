"""MCMC densification (Sec. Implementation: the densification of 3DGS replaced by the MCMC
approach of the cited work; appendix "Experimental Setup": densification every 100 iterations,
minimum opacity 0.1) -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may import
this module.  It shares no code with the HIP library.

The cited work is not part of the paper's text, so what follows is this repository's reading of
that method, restated in plain terms (every reading is also listed in the design notes):

* Gaussians are samples.  A *dead* Gaussian (opacity <= `dead_opacity`, the appendix's minimum
  opacity 0.1) is moved onto a live one drawn with probability proportional to opacity; *adding*
  Gaussians (up to a capacity, 5 % more per densification step) draws sources the same way and
  appends the copies.
* A source drawn c times ends up as N = c + 1 identical Gaussians (itself and its copies), with
  opacity o' = 1 - (1 - o)^(1/N) -- so the N copies stacked on one ray give the original opacity
  -- and scale s' = s o / S(N, o'),  S(N, a) = sum_{m=1..N} sum_{k=0..m-1} C(m-1, k) (-1)^k
  a^(k+1) / sqrt(k+1), which keeps the integral of the stacked copies' opacity profile along an
  axis equal to the original's.  N is capped at 51 in S and o' is kept in [0.005, 1 - 2^-23].
* Every Gaussian whose parameters are rewritten (the sources and their copies) restarts its Adam
  moments at zero.
* Between densification steps the means take Langevin noise: mu += lr_means * 5e5 *
  sigmoid(100 ((1 - o) - 0.995)) * Sigma eta, with eta ~ N(0, I) and Sigma = R diag(s^2) R^T.
* Two regularisers enter the loss: 0.01 mean(o) and 0.01 mean(s) over all scale entries.

Draws: the caller passes the random numbers in (one u32 per drawn sample, eta for the noise).
A draw r picks the source i whose integer weight interval [P_i, P_i + w_i) holds
t = floor(r * P / 2^32), with w_i = floor(o_i 2^24) (0 for a dead or non-live Gaussian) and P the
total: integer arithmetic, so both implementations take identical decisions.
"""
from __future__ import annotations

import math

import numpy as np

DEAD_OPACITY = 0.1
MIN_OPACITY = 0.005
N_MAX = 51
NOISE_LR = 5e5
GROWTH = 1.05
REG_OPACITY = 0.01
REG_SCALE = 0.01

f32 = np.float32


def weights(opacity: np.ndarray, n: int, dead_opacity: float = DEAD_OPACITY, live_only: bool = True) -> np.ndarray:
    """Integer sampling weights floor(o 2^24) of the first n Gaussians (0 for dead ones if live_only)."""
    o = np.asarray(opacity, np.float32)[:n]
    w = np.floor(o.astype(np.float64) * float(1 << 24)).astype(np.int64)
    if live_only:
        w[o <= f32(dead_opacity)] = 0
    return w


def draw(w: np.ndarray, r: np.ndarray) -> np.ndarray:
    """Sources for the u32 draws r: the i with P_i <= floor(r P / 2^32) < P_i + w_i (exact integers)."""
    P = int(w.sum())
    out = np.empty(len(r), np.int64)
    starts = np.concatenate([[0], np.cumsum(w)])
    for j, rj in enumerate(np.asarray(r, np.uint64)):
        t = (int(rj) * P) >> 32
        out[j] = int(np.searchsorted(starts, t, side="right")) - 1
    return out


def split_sum(N: int, a: float) -> float:
    """S(N, a) = sum_{m=1..N} sum_{k=0..m-1} C(m-1, k) (-1)^k a^(k+1) / sqrt(k+1), FP64."""
    s = 0.0
    for m in range(1, N + 1):
        for k in range(m):
            s += math.comb(m - 1, k) * (-1.0) ** k * a ** (k + 1) / math.sqrt(k + 1)
    return s


def split(o: float, s: np.ndarray, N: int):
    """Opacity and scales of each of N copies replacing one Gaussian (o, s)."""
    N = min(int(N), N_MAX)
    o_new = 1.0 - (1.0 - float(o)) ** (1.0 / N)
    o_new = min(max(o_new, MIN_OPACITY), 1.0 - 2.0 ** -23)
    f = float(o) / split_sum(N, o_new)
    return o_new, np.asarray(s, np.float64) * f


GROUPS = ("means", "log_scales", "quats", "logits", "sh")


def _rewrite(state: dict, sources: np.ndarray, dests: np.ndarray) -> dict:
    """Shared step of relocation and addition: split every drawn source, copy it to its destinations,
    zero the moments of every rewritten Gaussian.  state holds FP32 arrays [K][cap] per group (params,
    m_<group>, v_<group>) plus 'scales' and 'opacity' (activated copies)."""
    st = {k: np.array(v, copy=True) for k, v in state.items()}
    counts = np.bincount(sources, minlength=st["opacity"].shape[-1]) if len(sources) else \
        np.zeros(st["opacity"].shape[-1], np.int64)
    for i in np.nonzero(counts)[0]:
        o_new, s_new = split(st["opacity"][i], st["scales"][:, i], counts[i] + 1)
        st["opacity"][i] = f32(o_new)
        st["logits"][i] = f32(math.log(o_new / (1.0 - o_new)))
        st["scales"][:, i] = s_new.astype(np.float32)
        st["log_scales"][:, i] = np.log(s_new).astype(np.float32)
    touched = np.concatenate([np.nonzero(counts)[0], np.asarray(dests, np.int64)])
    for src, dst in zip(sources, dests):
        for g in GROUPS + ("scales", "opacity"):
            st[g][..., dst] = st[g][..., src]
    for g in GROUPS:
        st["m_" + g][..., touched] = 0.0
        st["v_" + g][..., touched] = 0.0
    return st


def relocate(state: dict, n: int, r: np.ndarray, dead_opacity: float = DEAD_OPACITY):
    """Move every dead Gaussian (index order) onto a live source drawn with r[j] (j = its dead rank).
    Returns (new state, dead indices, sources)."""
    o = np.asarray(state["opacity"], np.float32)[:n]
    dead = np.nonzero(o <= f32(dead_opacity))[0]
    w = weights(state["opacity"], n, dead_opacity, live_only=True)
    if len(dead) == 0 or w.sum() == 0:
        return {k: np.array(v, copy=True) for k, v in state.items()}, dead, np.zeros(0, np.int64)
    src = draw(w, np.asarray(r)[:len(dead)])
    return _rewrite(state, src, dead), dead, src


def add_count(n: int, cap: int, growth: float = GROWTH) -> int:
    """Gaussians added by one densification step: min(cap, floor(growth n)) - n, at least 0."""
    return max(0, min(int(cap), int(math.floor(growth * n))) - int(n))


def add(state: dict, n: int, cap: int, r: np.ndarray, growth: float = GROWTH):
    """Append add_count(n, cap) copies of sources drawn (over all n, by opacity) with r[j].
    Returns (new state, new n, sources)."""
    k = add_count(n, cap, growth)
    w = weights(state["opacity"], n, live_only=False)
    if k == 0 or w.sum() == 0:
        return {kk: np.array(v, copy=True) for kk, v in state.items()}, n, np.zeros(0, np.int64)
    src = draw(w, np.asarray(r)[:k])
    return _rewrite(state, src, np.arange(n, n + k)), n + k, src


def quat_to_rot(q: np.ndarray) -> np.ndarray:
    w, x, y, z = np.asarray(q, np.float64) / np.linalg.norm(q)
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def noise(means, scales, quats, opacity, eta, lr_means: float, n: int, noise_lr: float = NOISE_LR):
    """Means after the Langevin noise step (FP64)."""
    out = np.array(means, np.float64, copy=True)
    for i in range(n):
        R = quat_to_rot(quats[:, i])
        S = R @ np.diag(np.asarray(scales[:, i], np.float64) ** 2) @ R.T
        o = float(opacity[i])
        gate = 1.0 / (1.0 + math.exp(-100.0 * ((1.0 - o) - 0.995)))
        out[:, i] += lr_means * noise_lr * gate * (S @ np.asarray(eta[:, i], np.float64))
    return out


def reg_grads(n: int, lam_o: float = REG_OPACITY, lam_s: float = REG_SCALE):
    """Gradients of lam_o mean(o) + lam_s mean(s) w.r.t. each activated opacity and scale entry."""
    return lam_o / n, lam_s / (3.0 * n)
