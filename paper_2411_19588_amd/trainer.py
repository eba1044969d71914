"""A full training step over fixed views with every buffer allocated once.

forward (projection, depth-progressive binning, compositing with the medium)
-> L1 loss and its gradient -> adjoint -> Adam with the activation epilogue
(Sec. Optimization), all enqueued on one stream through the C ABI with fixed
pointers, so the whole step can be captured into a HIP graph and replayed.
With `fused=True` (what the benchmark trains with: faster on the 1M-Gaussian
1080p step) the Adam step runs inside the projection adjoint
(gs_render_backward_adam: the Gaussians' gradients never reach memory, and the
SH coefficients and means are stepped by a second kernel from the two factors
of their gradient); with `fused=False` the adjoint writes the gradients and
one flat Adam launch updates every group.  Raw parameters: means, log-scales,
quaternions, opacity logits, SH and the per-view medium coefficients.

The image loss is L1 (`loss="l1"`, the benchmark's) or eq. (OurFinalLoss)'s
(1 - lambda) L1 + lambda D-SSIM with lambda = 0.3 (`loss="l1_dssim"`, one fused
pass); with `prior_lambda > 0` the backward adds lambda_est L_best, pulling the
medium towards the backscatter estimates in `prior_est`, which
`estimate_backscatter()` recomputes from the targets and the last rendered depth
(every 500 iterations in the paper; outside any captured graph).  The MCMC
regularisers come from the rasterizer options (`reg_opacity`, `reg_scale`).

A step whose forward overflows the pair capacity is not applied: the device
training state (`state`, int32[2]: step counter, sticky skip flag) records it,
every later step is skipped too until `clear_skip()` (after the capacity has
been grown), so a replayed graph never updates the parameters from a truncated
render.  The same holds for a forward that `set_phase_limit()` cut short while a
tile was still unterminated (GS_STATUS_INCOMPLETE); `fit_phase_limit()` picks
the limit from a render with every phase, for replays of a fixed scene.
"""
from __future__ import annotations

import ctypes
import dataclasses
from typing import Optional, Sequence

import torch

from . import _native as N
from . import optim as OPT
from .rasterizer import RasterConfig, Rasterizer


def _vp(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


class TrainStep:
    def __init__(self, means, log_scales, quats, logits, sh, medium, sh_degree: int, cameras: Sequence,
                 targets: torch.Tensor, config: RasterConfig = RasterConfig(), max_pairs: Optional[int] = None,
                 lr: Optional[dict] = None, device="cuda", fused: bool = False, loss: str = "l1",
                 ssim_lambda: float = 0.3, prior_lambda: float = 0.0):
        dev = torch.device(device)
        lr = dict(OPT.LR, **(lr or {}))
        f32 = lambda t: t.to(dev, torch.float32).contiguous()
        self.groups = [OPT.Group("means", f32(means), lr["means"]),
                       OPT.Group("log_scales", f32(log_scales), lr["scales"], "exp"),
                       OPT.Group("quats", f32(quats), lr["quats"]),
                       OPT.Group("logits", f32(logits), lr["opacity"], "sigmoid"),
                       OPT.Group("sh", f32(sh), lr["sh"]),
                       OPT.Group("medium", f32(medium), lr["medium"])]
        self.G = {g.name: g for g in self.groups}
        self.fused = bool(fused)
        self.n = int(self.G["means"].param.shape[-1])
        self.sh_degree = int(sh_degree)
        self.rast = Rasterizer(cameras, config, device=dev)
        self.device = dev
        P = self.rast.total_pixels
        self.target = f32(targets).reshape(-1)
        if self.target.numel() != 3 * P:
            raise ValueError("targets must hold 3 * total pixels values (CHW per view, views packed)")
        self.rgb = torch.empty(3 * P, dtype=torch.float32, device=dev)
        self.depth = torch.empty(P, dtype=torch.float32, device=dev)
        self.alpha = torch.empty(P, dtype=torch.float32, device=dev)
        self.grad_rgb = torch.empty(3 * P, dtype=torch.float32, device=dev)
        self.loss = torch.empty(1, dtype=torch.float32, device=dev)
        self.state = torch.zeros(2, dtype=torch.int32, device=dev)   # (Adam step, sticky skip flag)
        self.graph = None
        self.timer = None
        if loss not in ("l1", "l1_dssim"):
            raise ValueError("loss must be 'l1' or 'l1_dssim'")
        self.loss_kind = loss
        self.ssim_lambda = float(ssim_lambda)
        self.loss_views = torch.empty(self.rast.n_views + 1, dtype=torch.float32, device=dev)
        self.loss_ws = None
        if loss == "l1_dssim":
            need = ctypes.c_size_t()
            N.check("gs_loss_workspace_query", N.lib().gs_loss_workspace_query(self.rast.n_views, self.rast.host_cams,
                                                                               ctypes.byref(need)))
            self.loss_ws = torch.empty(max(need.value, 256), dtype=torch.uint8, device=dev)
        # L_best: fixed buffer of the estimates (its address is baked into a captured graph)
        self.prior_lambda = float(prior_lambda)
        self.prior_est = torch.zeros(self.rast.n_views, 6, dtype=torch.float32, device=dev) \
            if self.prior_lambda > 0 else None
        self._estimator = None
        # A0: the groups hold the activated scales and opacities for the first forward (gs_activation)
        self._gauss = N.GsGaussians(self.n, self.sh_degree, 0, _vp(self.G["means"].param),
                                    _vp(self.G["log_scales"].activated), _vp(self.G["quats"].param),
                                    _vp(self.G["logits"].activated), _vp(self.G["sh"].param))
        self._grads = N.GsGaussianGrads(_vp(self.G["means"].grad), _vp(self.G["log_scales"].grad),
                                        _vp(self.G["quats"].grad), _vp(self.G["logits"].grad),
                                        _vp(self.G["sh"].grad))
        self._adam = (N.GsAdamGroup * len(self.groups))()
        for i, g in enumerate(self.groups):
            self._adam[i] = N.GsAdamGroup(g.param.data_ptr(), g.grad.data_ptr(), g.m.data_ptr(), g.v.data_ptr(),
                                          g.activated.data_ptr() if g.activated is not None else None,
                                          g.param.numel(), g.lr, OPT._ACT[g.activation], 0)
        self.set_capacity(max_pairs if max_pairs is not None else config.max_pairs)

    # ------------------------------------------------------------------ buffers
    def set_capacity(self, max_pairs: int) -> None:
        """(Re)allocate the workspace and forward context for `max_pairs` stored pairs (drops any graph)."""
        self.destroy_graph()
        self.max_pairs = int(max_pairs)
        self.opts = self.rast.config.to_c(self.max_pairs, None, self.prior_est, self.prior_lambda)
        ws, sv = self.rast.sizes_for(self.n, self.max_pairs)
        self.ws = torch.empty(max(ws, 256), dtype=torch.uint8, device=self.device)
        self.saved = torch.empty(max(sv, 256), dtype=torch.uint8, device=self.device)

    def estimate_backscatter(self, cfg=None) -> torch.Tensor:
        """Recompute prior_est (Alg. 1 and Alg. 2) from the targets and the depth of the last forward."""
        if self.prior_est is None:
            raise RuntimeError("construct the step with prior_lambda > 0 to use the backscatter prior")
        from .backscatter import BackscatterEstimator
        if self._estimator is None or cfg is not None:
            self._estimator = BackscatterEstimator(self.rast, cfg)
        self.prior_est.copy_(self._estimator(self.target, self.depth))
        return self.prior_est

    def size_capacity(self, headroom: float = 1.25) -> int:
        """Run one eager forward (growing the capacity until it fits) and leave `headroom` over its need."""
        s = torch.cuda.current_stream(self.device)
        while True:
            self._forward(s)
            st, need = self.rast.read_status(self.saved, s)
            if st & N.GS_STATUS_PAIR_OVERFLOW:
                self.set_capacity(min(N.GS_MAX_PAIRS, int(need * headroom) + 4096))
                continue
            break
        want = min(N.GS_MAX_PAIRS, int(need * headroom) + 4096)
        if want > self.max_pairs:
            self.set_capacity(want)
        return need

    # ------------------------------------------------------------------ depth phases
    def set_phase_limit(self, limit: int) -> None:
        """Run only the first `limit` depth phases of the schedule (0 = all; drops any graph).  A
        forward that the limit cuts short while a tile is unterminated and Gaussians are left
        unbinned reports GS_STATUS_INCOMPLETE: its step is not applied and the sticky skip flag is
        set, as after a pair-capacity overflow."""
        self.destroy_graph()
        self.rast.config = dataclasses.replace(self.rast.config, phase_limit=int(limit))
        self.opts.phase_limit = int(limit)

    def fit_phase_limit(self) -> int:
        """Render once with every phase, then run only the leading phases that render needed
        (gs_phases_needed): for replays of a fixed scene, the same images without the launches of
        phases that would blend nothing.  Returns the limit."""
        self.set_phase_limit(0)
        s = torch.cuda.current_stream(self.device)
        self._forward(s)
        st, _ = self.rast.read_status(self.saved, s)
        if st & N.GS_STATUS_PAIR_OVERFLOW:
            raise RuntimeError("the forward overflowed the pair capacity: call size_capacity() first")
        k = self.rast.phases_needed(self.saved, self.n, self.max_pairs, s)
        self.set_phase_limit(k)
        return k

    # ------------------------------------------------------------------ step
    def _forward(self, stream) -> None:
        sp = ctypes.c_void_p(stream.cuda_stream)
        self.opts.timer = self.timer
        N.check("gs_render_forward", N.lib().gs_render_forward(
            ctypes.byref(self.opts), ctypes.byref(self._gauss), self.rast.n_views, self.rast.host_cams,
            _vp(self.rast.dev_cams), _vp(self.G["medium"].param), _vp(self.rgb), _vp(self.depth), _vp(self.alpha),
            None, _vp(self.saved), self.saved.numel(), _vp(self.ws), self.ws.numel(), sp))

    def enqueue(self, stream=None) -> None:
        """Enqueue one training step on `stream` (no host synchronisation)."""
        stream = torch.cuda.current_stream(self.device) if stream is None else stream
        sp = ctypes.c_void_p(stream.cuda_stream)
        L = N.lib()
        self._forward(stream)
        if self.loss_kind == "l1":
            N.check("gs_l1_loss", L.gs_l1_loss(self.rgb.numel(), _vp(self.rgb), _vp(self.target), _vp(self.loss),
                                               _vp(self.grad_rgb), sp))
        else:
            N.check("gs_l1_dssim_loss", L.gs_l1_dssim_loss(
                self.rast.n_views, self.rast.host_cams, _vp(self.rgb), _vp(self.target), self.ssim_lambda,
                _vp(self.loss_views), _vp(self.grad_rgb), _vp(self.loss_ws), self.loss_ws.numel(), sp))
        if self.fused:
            N.check("gs_render_backward_adam", L.gs_render_backward_adam(
                ctypes.byref(self.opts), ctypes.byref(self._gauss), self.rast.n_views, self.rast.host_cams,
                _vp(self.rast.dev_cams), _vp(self.G["medium"].param), _vp(self.grad_rgb), None, None,
                _vp(self.saved), self.saved.numel(), self._adam, 0.9, 0.999, 1e-8, _vp(self.state), _vp(self.ws),
                self.ws.numel(), sp))
            return
        N.check("gs_render_backward", L.gs_render_backward(
            ctypes.byref(self.opts), ctypes.byref(self._gauss), self.rast.n_views, self.rast.host_cams,
            _vp(self.rast.dev_cams), _vp(self.G["medium"].param), _vp(self.grad_rgb), None, None, _vp(self.saved),
            self.saved.numel(), ctypes.byref(self._grads), _vp(self.G["medium"].grad), _vp(self.ws),
            self.ws.numel(), sp))
        N.check("gs_adam_step_device", L.gs_adam_step_device(self._adam, len(self.groups), 0.9, 0.999, 1e-8,
                                                             _vp(self.state), _vp(self.saved), sp))

    # ------------------------------------------------------------------ training state
    @property
    def step_counter(self) -> torch.Tensor:
        """The device Adam step counter (a view of state[0])."""
        return self.state[N.GS_STATE_STEP:N.GS_STATE_STEP + 1]

    def skipped(self) -> int:
        """Sticky skip flag (GS_STATUS_* bits of the overflow that stopped the updates; synchronises)."""
        return int(self.state[N.GS_STATE_SKIP].item())

    def clear_skip(self) -> None:
        """Let steps apply again (after the capacity has been grown to what the forward needs)."""
        self.state[N.GS_STATE_SKIP].zero_()

    # ------------------------------------------------------------------ graph
    def capture(self, stream: torch.cuda.Stream) -> None:
        """Capture one step into a HIP graph on `stream` (a non-default stream)."""
        self.destroy_graph()
        if self.timer is not None:
            raise RuntimeError("disable the timer while capturing")
        sp = ctypes.c_void_p(stream.cuda_stream)
        g = ctypes.c_void_p()
        N.check("gs_graph_begin", N.lib().gs_graph_begin(sp))
        try:
            self.enqueue(stream)
        finally:
            rc = N.lib().gs_graph_end(sp, ctypes.byref(g))
        N.check("gs_graph_end", rc)
        self.graph = g

    def replay(self, stream: torch.cuda.Stream) -> None:
        N.check("gs_graph_launch", N.lib().gs_graph_launch(self.graph, ctypes.c_void_p(stream.cuda_stream)))

    def destroy_graph(self) -> None:
        if getattr(self, "graph", None) is not None:
            N.lib().gs_graph_destroy(self.graph)
            self.graph = None

    def status(self, stream=None):
        return self.rast.read_status(self.saved, stream)

    def __del__(self):
        try:
            self.destroy_graph()
        except Exception:
            pass


class RenderStep:
    """Forward + L1 loss + backward over a fixed camera list with every buffer allocated once.

    Parameters are taken as given (activated scales and opacities); gradients land in
    `self.grads` and `self.grad_medium` (overwritten each step, summed over the views
    inside the library).  Graph-capturable like TrainStep.  Used by the autotuner and to
    time a batch of views rendered by one pipeline against one pipeline per view.
    """

    def __init__(self, params: dict, sh_degree: int, cameras: Sequence, medium: torch.Tensor, targets: torch.Tensor,
                 config: RasterConfig = RasterConfig(), max_pairs: Optional[int] = None,
                 grad_medium: Optional[torch.Tensor] = None, device="cuda"):
        dev = torch.device(device)
        self.device = dev
        self.p = params
        self.n = int(params["means"].shape[-1])
        self.sh_degree = int(sh_degree)
        self.rast = Rasterizer(cameras, config, device=dev)
        self.medium = medium
        P = self.rast.total_pixels
        self.target = targets.reshape(-1)
        if self.target.numel() != 3 * P:
            raise ValueError("targets must hold 3 * total pixels values")
        self.rgb = torch.empty(3 * P, dtype=torch.float32, device=dev)
        self.depth = torch.empty(P, dtype=torch.float32, device=dev)
        self.alpha = torch.empty(P, dtype=torch.float32, device=dev)
        self.grad_rgb = torch.empty(3 * P, dtype=torch.float32, device=dev)
        self.loss = torch.empty(1, dtype=torch.float32, device=dev)
        self.grads = {k: torch.empty_like(params[k]) for k in ("means", "scales", "quats", "opacity", "sh")}
        self.grad_medium = torch.empty(self.rast.n_views * 9, dtype=torch.float32, device=dev) \
            if grad_medium is None else grad_medium
        self.graph = None
        self._gauss = N.GsGaussians(self.n, self.sh_degree, 0, *(_vp(params[k]) for k in
                                                                 ("means", "scales", "quats", "opacity", "sh")))
        self._grads = N.GsGaussianGrads(*(_vp(self.grads[k]) for k in ("means", "scales", "quats", "opacity", "sh")))
        self.set_capacity(max_pairs if max_pairs is not None else config.max_pairs)

    def set_capacity(self, max_pairs: int) -> None:
        self.destroy_graph()
        self.max_pairs = int(max_pairs)
        self.opts = self.rast.config.to_c(self.max_pairs)
        ws, sv = self.rast.sizes_for(self.n, self.max_pairs)
        self.ws = torch.empty(max(ws, 256), dtype=torch.uint8, device=self.device)
        self.saved = torch.empty(max(sv, 256), dtype=torch.uint8, device=self.device)

    def size_capacity(self, headroom: float = 1.25) -> int:
        s = torch.cuda.current_stream(self.device)
        while True:
            self._forward(s)
            st, need = self.rast.read_status(self.saved, s)
            if st & N.GS_STATUS_PAIR_OVERFLOW:
                self.set_capacity(min(N.GS_MAX_PAIRS, int(need * headroom) + 4096))
                continue
            break
        want = min(N.GS_MAX_PAIRS, int(need * headroom) + 4096)
        if want > self.max_pairs:
            self.set_capacity(want)
        return need

    def _forward(self, stream) -> None:
        N.check("gs_render_forward", N.lib().gs_render_forward(
            ctypes.byref(self.opts), ctypes.byref(self._gauss), self.rast.n_views, self.rast.host_cams,
            _vp(self.rast.dev_cams), _vp(self.medium), _vp(self.rgb), _vp(self.depth), _vp(self.alpha), None,
            _vp(self.saved), self.saved.numel(), _vp(self.ws), self.ws.numel(), ctypes.c_void_p(stream.cuda_stream)))

    def enqueue(self, stream=None) -> None:
        stream = torch.cuda.current_stream(self.device) if stream is None else stream
        sp = ctypes.c_void_p(stream.cuda_stream)
        L = N.lib()
        self._forward(stream)
        N.check("gs_l1_loss", L.gs_l1_loss(self.rgb.numel(), _vp(self.rgb), _vp(self.target), _vp(self.loss),
                                           _vp(self.grad_rgb), sp))
        N.check("gs_render_backward", L.gs_render_backward(
            ctypes.byref(self.opts), ctypes.byref(self._gauss), self.rast.n_views, self.rast.host_cams,
            _vp(self.rast.dev_cams), _vp(self.medium), _vp(self.grad_rgb), None, None, _vp(self.saved),
            self.saved.numel(), ctypes.byref(self._grads), _vp(self.grad_medium), _vp(self.ws), self.ws.numel(),
            sp))

    def capture(self, stream: torch.cuda.Stream) -> None:
        self.destroy_graph()
        sp = ctypes.c_void_p(stream.cuda_stream)
        g = ctypes.c_void_p()
        N.check("gs_graph_begin", N.lib().gs_graph_begin(sp))
        try:
            self.enqueue(stream)
        finally:
            rc = N.lib().gs_graph_end(sp, ctypes.byref(g))
        N.check("gs_graph_end", rc)
        self.graph = g

    def replay(self, stream: torch.cuda.Stream) -> None:
        N.check("gs_graph_launch", N.lib().gs_graph_launch(self.graph, ctypes.c_void_p(stream.cuda_stream)))

    def destroy_graph(self) -> None:
        if getattr(self, "graph", None) is not None:
            N.lib().gs_graph_destroy(self.graph)
            self.graph = None

    def status(self, stream=None):
        return self.rast.read_status(self.saved, stream)

    def __del__(self):
        try:
            self.destroy_graph()
        except Exception:
            pass
