"""PyTorch front end of libgsplash: buffers, streams and autograd.

Every computation happens in the HIP library; this module only allocates
device memory with torch, passes pointers and the current HIP stream, and
wires gs_render_forward / gs_render_backward into ``torch.autograd``.
"""
from __future__ import annotations

import ctypes
import dataclasses
from typing import List, Optional, Sequence, Tuple

import torch

from . import _native as N


@dataclasses.dataclass
class RasterConfig:
    """Rasterizer options (gs_options).  Defaults follow the readings of the
    discrete rules the paper inherits from 3DGS: alpha skip 1/255, alpha clamp
    0.99, termination at T < 1e-4, EWA dilation 0.3, extent kappa 11.1."""
    tile: int = 16
    lds_batch: int = 64
    persistent: int = 0               # 0 one workgroup per tile; 1 persistent queue; 2 longest list first
    pixels_per_lane: int = 0          # 0 = library default
    record_fetch: str = "default"     # "default", "lds" or "scalar"
    alpha_min: float = 1.0 / 255.0
    alpha_max: float = 0.99
    t_min: float = 1e-4
    dilation: float = 0.3
    kappa: float = 11.1
    depth_mode: int = 0               # z of the medium term: 0 metric, 1 logistic map
    depth_output: int = 0             # depth image: 0 the medium's z, 1 the logistic map (visualisation)
    tile_cull: bool = True            # drop (Gaussian, tile) pairs that cannot reach alpha_min
    phases: int = 0                   # 0 = automatic (the library's gs_schedule)
    phase0_shift: int = 0             # 0 = automatic
    phase_growth: int = 0             # log2 of the later phases' growth; 0 = automatic (4x)
    phase_limit: int = 0              # run only the first phase_limit depth phases (0 = all); a forward
                                      # left with an unterminated tile and unbinned Gaussians reports
                                      # GS_STATUS_INCOMPLETE
    max_pairs: int = 1 << 22
    reg_opacity: float = 0.0          # lambda_o of the opacity regulariser lambda_o mean(o) (0 = off)
    reg_scale: float = 0.0            # lambda_s of the scale regulariser lambda_s mean(s) (0 = off)

    def to_c(self, max_pairs: Optional[int] = None, timer=None, prior: Optional[torch.Tensor] = None,
             prior_lambda: float = 0.0) -> N.GsOptions:
        o = N.default_options()
        o.tile_w = o.tile_h = int(self.tile)
        o.lds_batch = int(self.lds_batch)
        o.persistent = int(self.persistent)
        o.pixels_per_lane = int(self.pixels_per_lane)
        o.record_fetch = {"default": N.GS_FETCH_DEFAULT, "lds": N.GS_FETCH_LDS,
                          "scalar": N.GS_FETCH_SCALAR}[self.record_fetch]
        o.alpha_min = self.alpha_min
        o.alpha_max = self.alpha_max
        o.t_min = self.t_min
        o.dilation = self.dilation
        o.kappa = self.kappa
        o.depth_mode = int(self.depth_mode)
        o.depth_output = int(self.depth_output)
        o.tile_cull = 1 if self.tile_cull else 0
        o.phases = int(self.phases)
        o.phase0_shift = int(self.phase0_shift)
        o.phase_growth = int(self.phase_growth)
        o.phase_limit = int(self.phase_limit)
        o.max_pairs = int(self.max_pairs if max_pairs is None else max_pairs)
        o.timer = timer
        o.reg_opacity = float(self.reg_opacity)
        o.reg_scale = float(self.reg_scale)
        if prior is not None:
            if prior.dtype != torch.float32 or not prior.is_contiguous():
                raise ValueError("the medium prior must be a contiguous float32 [views, 6] tensor")
            o.medium_prior = prior.data_ptr()
            o.prior_lambda = float(prior_lambda)
        return o


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream=None) -> ctypes.c_void_p:
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _f32(t: torch.Tensor) -> torch.Tensor:
    if t.dtype != torch.float32 or not t.is_contiguous():
        t = t.to(torch.float32).contiguous()
    return t


@dataclasses.dataclass
class ForwardContext:
    saved: torch.Tensor
    max_pairs: int
    n: int
    sh_degree: int
    # the cameras of this forward (a device copy and the host array): the adjoint must see the
    # poses the forward used even if the rasterizer's cameras are changed in between
    dev_cams: Optional[torch.Tensor] = None
    host_cams: Optional[ctypes.Array] = None
    restored: Optional[torch.Tensor] = None   # the clean image J = C_air, when requested


class Rasterizer:
    """Renders Gaussians into a fixed set of views (sizes fixed; poses may change).

    Views are packed: view v's pixels start at ``pixel_offsets[v]``; ``rgb``
    is [3 * total_pixels] with a CHW plane per view.
    """

    def __init__(self, cameras: Sequence, config: RasterConfig = RasterConfig(), device="cuda"):
        if len(cameras) < 1 or len(cameras) > N.GS_MAX_VIEWS:
            raise ValueError(f"1..{N.GS_MAX_VIEWS} views supported")
        self.config = config
        self.device = torch.device(device)
        self.host_cams = N.camera_array(cameras)
        self.n_views = len(cameras)
        self.sizes = [(int(c.width), int(c.height)) for c in cameras]
        offs = [0]
        for w, h in self.sizes:
            offs.append(offs[-1] + w * h)
        self.pixel_offsets = offs
        self.total_pixels = offs[-1]
        self.dev_cams = torch.empty(ctypes.sizeof(self.host_cams), dtype=torch.uint8, device=self.device)
        self.set_cameras(cameras)
        self.max_pairs = int(config.max_pairs)
        self._ws: Optional[torch.Tensor] = None
        self.timer = None
        # L_best of eq. (OurFinalLoss): [views, 6] estimates (B_inf_hat, B_b_hat) the backward pulls
        # the medium towards with weight prior_lambda (None = no prior)
        self.medium_prior: Optional[torch.Tensor] = None
        self.prior_lambda = 0.0

    # ---------------------------------------------------------------- cameras
    def set_cameras(self, cameras: Sequence) -> None:
        """Update the device copy of the poses/intrinsics in place (sizes must not change)."""
        arr = N.camera_array(cameras)
        for i, c in enumerate(cameras):
            if (int(c.width), int(c.height)) != self.sizes[i]:
                raise ValueError("view sizes are fixed for a Rasterizer")
        self.host_cams = arr
        buf = torch.frombuffer(bytearray(bytes(arr)), dtype=torch.uint8)
        self.dev_cams.copy_(buf, non_blocking=False)

    def tile_count(self) -> int:
        return int(N.lib().gs_tile_count(ctypes.byref(self.config.to_c()), self.n_views, self.host_cams))

    def schedule(self, n: int):
        """(phases, phase0_shift) the library uses for n Gaussians, this configuration and these views."""
        p, sh = ctypes.c_int32(), ctypes.c_int32()
        N.check("gs_schedule", N.lib().gs_schedule(ctypes.byref(self.config.to_c()), int(n), self.n_views,
                                                   self.host_cams, ctypes.byref(p), ctypes.byref(sh)))
        return p.value, sh.value

    # ---------------------------------------------------------------- buffers
    def sizes_for(self, n: int, max_pairs: int) -> Tuple[int, int]:
        ws = ctypes.c_size_t()
        sv = ctypes.c_size_t()
        o = self.config.to_c(max_pairs)
        N.check("gs_workspace_query", N.lib().gs_workspace_query(ctypes.byref(o), n, self.n_views, self.host_cams,
                                                                 ctypes.byref(ws), ctypes.byref(sv)))
        return ws.value, sv.value

    def workspace(self, nbytes: int) -> torch.Tensor:
        if self._ws is None or self._ws.numel() < nbytes:
            self._ws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=self.device)
        return self._ws

    # ---------------------------------------------------------------- forward / backward
    def _gaussians(self, means, scales, quats, opacity, sh, sh_degree) -> N.GsGaussians:
        n = means.shape[-1]
        return N.GsGaussians(n, sh_degree, 0, _ptr(means), _ptr(scales), _ptr(quats), _ptr(opacity), _ptr(sh))

    def forward(self, means, scales, quats, opacity, sh, sh_degree: int, medium: torch.Tensor,
                check: bool = True, max_pairs: Optional[int] = None, stream=None, restored: bool = False):
        """Render all views.  Returns (rgb, depth, alpha, ForwardContext).

        With check=True the status word is read after the forward (one host
        synchronisation); on pair-capacity overflow the capacity is grown to
        what the forward needed and the render is repeated, and a render that
        config.phase_limit cut short is repeated with every phase.  With restored=True
        the clean image J = C_air (packed like rgb) is returned in ctx.restored.
        """
        means, scales, quats, opacity, sh = map(_f32, (means, scales, quats, opacity, sh))
        medium = _f32(medium)
        n = int(means.shape[-1])
        mp = int(self.max_pairs if max_pairs is None else max_pairs)
        L = N.lib()
        g = self._gaussians(means, scales, quats, opacity, sh, sh_degree)
        full = False   # set after a forward that config.phase_limit cut short: render every phase
        while True:
            ws_b, sv_b = self.sizes_for(n, mp)
            ws = self.workspace(ws_b)
            saved = torch.empty(sv_b, dtype=torch.uint8, device=self.device)
            rgb = torch.empty(3 * self.total_pixels, dtype=torch.float32, device=self.device)
            depth = torch.empty(self.total_pixels, dtype=torch.float32, device=self.device)
            alpha = torch.empty(self.total_pixels, dtype=torch.float32, device=self.device)
            rest = torch.empty(3 * self.total_pixels, dtype=torch.float32, device=self.device) if restored else None
            o = self.config.to_c(mp, self.timer)
            if full:
                o.phase_limit = 0
            N.check("gs_render_forward", L.gs_render_forward(
                ctypes.byref(o), ctypes.byref(g), self.n_views, self.host_cams, _ptr(self.dev_cams), _ptr(medium),
                _ptr(rgb), _ptr(depth), _ptr(alpha), _ptr(rest), _ptr(saved), sv_b, _ptr(ws), ws_b,
                _stream(stream)))
            if not check:
                break
            status, needed = self.read_status(saved, stream)
            if status & N.GS_STATUS_PAIR_OVERFLOW:
                if needed > N.GS_MAX_PAIRS:
                    raise RuntimeError(f"{needed} (Gaussian, tile) pairs exceed the 32-bit pair index")
                mp = min(N.GS_MAX_PAIRS, int(needed * 1.25) + 1024)
                self.max_pairs = mp
                continue
            if status & N.GS_STATUS_INCOMPLETE:
                full = True
                continue
            break
        host_copy = (N.GsCamera * self.n_views)()
        ctypes.memmove(host_copy, self.host_cams, ctypes.sizeof(host_copy))
        return rgb, depth, alpha, ForwardContext(saved, mp, n, sh_degree, self.dev_cams.clone(), host_copy, rest)

    def backward(self, ctx: ForwardContext, means, scales, quats, opacity, sh, medium, grad_rgb,
                 grad_depth=None, stream=None, out=None, grad_restored=None):
        """Adjoint of forward(); returns (d_means, d_scales, d_quats, d_opacity, d_sh, d_medium).

        The cameras are those the forward used (kept in `ctx`).  `out` may supply those six
        tensors (contiguous float32, same shapes) to be overwritten.  grad_restored is the
        upstream gradient of the clean image J (packed like rgb), or None.
        """
        means, scales, quats, opacity, sh = map(_f32, (means, scales, quats, opacity, sh))
        medium = _f32(medium)
        grad_rgb = _f32(grad_rgb)
        grad_depth = None if grad_depth is None else _f32(grad_depth)
        grad_restored = None if grad_restored is None else _f32(grad_restored)
        host_cams = self.host_cams if ctx.host_cams is None else ctx.host_cams
        dev_cams = self.dev_cams if ctx.dev_cams is None else ctx.dev_cams
        n = ctx.n
        ws_b, sv_b = self.sizes_for(n, ctx.max_pairs)
        ws = self.workspace(ws_b)
        if out is not None:
            *outs, gmed = out
            for o_, ref in zip(outs + [gmed], (means, scales, quats, opacity, sh, medium)):
                if o_.dtype != torch.float32 or not o_.is_contiguous() or o_.numel() != ref.numel():
                    raise ValueError("gradient buffers must be contiguous float32 of the parameter sizes")
        else:
            outs = [torch.empty_like(t) for t in (means, scales, quats, opacity, sh)]
            gmed = torch.empty((self.n_views, 9), dtype=torch.float32, device=self.device)
        g = self._gaussians(means, scales, quats, opacity, sh, ctx.sh_degree)
        grads = N.GsGaussianGrads(*[_ptr(t) for t in outs])
        o = self.config.to_c(ctx.max_pairs, self.timer, self.medium_prior, self.prior_lambda)
        N.check("gs_render_backward", N.lib().gs_render_backward(
            ctypes.byref(o), ctypes.byref(g), self.n_views, host_cams, _ptr(dev_cams), _ptr(medium),
            _ptr(grad_rgb), _ptr(grad_depth), _ptr(grad_restored), _ptr(ctx.saved), sv_b, ctypes.byref(grads),
            _ptr(gmed), _ptr(ws), ws_b, _stream(stream)))
        return (*outs, gmed)

    def read_status(self, saved: torch.Tensor, stream=None) -> Tuple[int, int]:
        st = ctypes.c_uint32()
        need = ctypes.c_int64()
        N.check("gs_read_status", N.lib().gs_read_status(_ptr(saved), ctypes.byref(st), ctypes.byref(need),
                                                         _stream(stream)))
        return int(st.value), int(need.value)

    def phases_needed(self, saved: torch.Tensor, n: int, max_pairs: int, stream=None) -> int:
        """Leading depth phases the forward that wrote `saved` needed (gs_phases_needed; synchronises)."""
        k = ctypes.c_int32()
        o = self.config.to_c(max_pairs)
        N.check("gs_phases_needed", N.lib().gs_phases_needed(ctypes.byref(o), int(n), self.n_views, self.host_cams,
                                                             _ptr(saved), saved.numel(), ctypes.byref(k),
                                                             _stream(stream)))
        return int(k.value)

    def export_keys(self, ctx: ForwardContext, stream=None):
        """Stored (tile << 32 | depth bits) keys, values (view * n + index) and per-phase tile ranges
        [GS_MAX_PHASES, tiles, 2] of a forward (one sorted run per phase)."""
        T = self.tile_count()
        cap = ctx.max_pairs
        keys = torch.empty(max(cap, 1), dtype=torch.int64, device=self.device)
        vals = torch.empty(max(cap, 1), dtype=torch.int32, device=self.device)
        ranges = torch.empty(max(2 * T * N.GS_MAX_PHASES, 2), dtype=torch.int32, device=self.device)
        cnt = ctypes.c_int64()
        o = self.config.to_c(ctx.max_pairs)
        N.check("gs_export_keys", N.lib().gs_export_keys(
            ctypes.byref(o), ctx.n, self.n_views, self.host_cams, _ptr(ctx.saved), ctx.saved.numel(), _ptr(keys),
            _ptr(vals), _ptr(ranges), cap, ctypes.byref(cnt), _stream(stream)))
        k = int(cnt.value)
        return keys[:k], vals[:k], ranges[: 2 * T * N.GS_MAX_PHASES].view(N.GS_MAX_PHASES, T, 2)

    def forward_stats(self, ctx: ForwardContext, stream=None):
        """(K pairs, E walked list entries, list entries reached, non-empty tiles, blended evaluations)."""
        st = (ctypes.c_int64 * 5)()
        o = self.config.to_c(ctx.max_pairs)
        N.check("gs_forward_stats", N.lib().gs_forward_stats(ctypes.byref(o), ctx.n, self.n_views, self.host_cams,
                                                             _ptr(ctx.saved), ctx.saved.numel(), st,
                                                             _stream(stream)))
        return tuple(int(x) for x in st)

    # ---------------------------------------------------------------- views
    def split(self, rgb: torch.Tensor, depth: torch.Tensor, alpha: torch.Tensor):
        """Per-view (rgb (3,H,W), depth (H,W), alpha (H,W)) views of the packed outputs."""
        out = []
        for v, (w, h) in enumerate(self.sizes):
            p0 = self.pixel_offsets[v]
            out.append((rgb[3 * p0: 3 * p0 + 3 * w * h].view(3, h, w), depth[p0: p0 + w * h].view(h, w),
                        alpha[p0: p0 + w * h].view(h, w)))
        return out


class _RenderFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, means, scales, quats, opacity, sh, medium, rast: Rasterizer, sh_degree: int,
                restored: bool = False):
        rgb, depth, alpha, fctx = rast.forward(means, scales, quats, opacity, sh, sh_degree, medium,
                                               restored=restored)
        ctx.save_for_backward(means, scales, quats, opacity, sh, medium)
        ctx.rast = rast
        ctx.fctx = fctx
        ctx.mark_non_differentiable(alpha)
        if restored:
            return rgb, depth, alpha, fctx.restored
        return rgb, depth, alpha

    @staticmethod
    def backward(ctx, g_rgb, g_depth, g_alpha, g_restored=None):
        means, scales, quats, opacity, sh, medium = ctx.saved_tensors
        if g_rgb is None:
            g_rgb = torch.zeros(3 * ctx.rast.total_pixels, dtype=torch.float32, device=means.device)
        gm, gs_, gq, go, gsh, gmed = ctx.rast.backward(ctx.fctx, means, scales, quats, opacity, sh, medium,
                                                       g_rgb, g_depth, grad_restored=g_restored)
        return gm, gs_, gq, go, gsh, gmed.view_as(medium), None, None, None


class _ActivateFn(torch.autograd.Function):
    """exp(log-scale), sigmoid(logit) via gs_activate / gs_activate_backward."""

    @staticmethod
    def forward(ctx, log_scales, logits):
        log_scales = _f32(log_scales)
        logits = _f32(logits)
        n = int(logits.shape[-1])
        s = torch.empty_like(log_scales)
        o = torch.empty_like(logits)
        N.check("gs_activate", N.lib().gs_activate(n, _ptr(log_scales), _ptr(logits), _ptr(s), _ptr(o), _stream()))
        ctx.save_for_backward(s, o)
        return s, o

    @staticmethod
    def backward(ctx, g_s, g_o):
        s, o = ctx.saved_tensors
        g_s = torch.zeros_like(s) if g_s is None else _f32(g_s)
        g_o = torch.zeros_like(o) if g_o is None else _f32(g_o)
        gls = torch.empty_like(s)
        glg = torch.empty_like(o)
        n = int(o.shape[-1])
        N.check("gs_activate_backward", N.lib().gs_activate_backward(
            n, _ptr(s), _ptr(o), _ptr(g_s), _ptr(g_o), _ptr(gls), _ptr(glg), _stream()))
        return gls, glg


def activate(log_scales: torch.Tensor, logits: torch.Tensor):
    """Differentiable (scales, opacity) = (exp(log_scales), sigmoid(logits)) on the GPU."""
    return _ActivateFn.apply(log_scales, logits)


def render(means, scales, quats, opacity, sh, medium, rast: Rasterizer, sh_degree: int, restored: bool = False):
    """Differentiable render of all views of `rast`.

    means [3,N], scales [3,N] (activated), quats [4,N], opacity [N] (activated),
    sh [(deg+1)^2*3, N], medium [V,9].  Returns packed (rgb, depth, alpha), and with
    restored=True also the clean image J = C_air (packed like rgb, eq. scattering_approx);
    gradients flow from every output but alpha (non-differentiable) to every input.
    """
    return _RenderFn.apply(means, scales, quats, opacity, sh, medium, rast, sh_degree, restored)


def l1_loss(pred: torch.Tensor, target: torch.Tensor, with_loss: bool = True):
    """(loss [1] or None, grad) of mean |pred - target| via gs_l1_loss."""
    pred = _f32(pred)
    target = _f32(target)
    grad = torch.empty_like(pred)
    loss = torch.empty(1, dtype=torch.float32, device=pred.device) if with_loss else None
    N.check("gs_l1_loss", N.lib().gs_l1_loss(pred.numel(), _ptr(pred), _ptr(target), _ptr(loss), _ptr(grad),
                                              _stream()))
    return loss, grad


def l1_dssim_loss(pred: torch.Tensor, target: torch.Tensor, rast: Rasterizer, lam: float = 0.3,
                  with_loss: bool = True, workspace: Optional[torch.Tensor] = None):
    """(loss [V + 1] or None, grad) of sum_v (1 - lam) L1_v + lam D-SSIM_v via gs_l1_dssim_loss.

    pred and target are packed like the rasterizer's rgb output; loss holds each view's term and
    then their sum (eq. 3DGSoriginalLoss with lambda = 0.3 in the paper)."""
    pred = _f32(pred)
    target = _f32(target)
    L = N.lib()
    need = ctypes.c_size_t()
    N.check("gs_loss_workspace_query", L.gs_loss_workspace_query(rast.n_views, rast.host_cams, ctypes.byref(need)))
    if workspace is None or workspace.numel() < need.value:
        workspace = torch.empty(max(need.value, 256), dtype=torch.uint8, device=pred.device)
    grad = torch.empty_like(pred)
    loss = torch.empty(rast.n_views + 1, dtype=torch.float32, device=pred.device) if with_loss else None
    N.check("gs_l1_dssim_loss", L.gs_l1_dssim_loss(rast.n_views, rast.host_cams, _ptr(pred), _ptr(target), float(lam),
                                                   _ptr(loss), _ptr(grad), _ptr(workspace), workspace.numel(),
                                                   _stream()))
    return loss, grad
