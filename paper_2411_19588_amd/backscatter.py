"""PyTorch front end of the backscatter estimation (Sec. Optimization; appendix "Backscatter
Estimation", Alg. 1 and Alg. 2) and of the L_best prior of eq. (OurFinalLoss).

Argument marshalling only: gs_estimate_backscatter and gs_backscatter_prior do the work.
"""
from __future__ import annotations

import ctypes
import dataclasses
from typing import Optional, Tuple

import torch

from . import _native as N
from .rasterizer import Rasterizer, _f32, _ptr, _stream


@dataclasses.dataclass
class BackscatterConfig:
    """Alg. 1 / Alg. 2 inputs: p_dark 0.01, 10 cluster edges, 25 interval edges, 300 rows."""
    p_dark: float = 0.01
    edges: int = 10
    intervals: int = 25
    resize_height: int = 300

    def to_c(self) -> N.GsBackscatterOptions:
        o = N.GsBackscatterOptions()
        N.lib().gs_default_backscatter_options(ctypes.byref(o))
        o.p_dark = float(self.p_dark)
        o.edges = int(self.edges)
        o.intervals = int(self.intervals)
        o.resize_height = int(self.resize_height)
        return o


class BackscatterEstimator:
    """Estimates (B_inf_hat, B_b_hat) per view of a rasterizer's views; keeps its workspace."""

    def __init__(self, rast: Rasterizer, cfg: Optional[BackscatterConfig] = None):
        self.rast = rast
        self.cfg = cfg or BackscatterConfig()
        self.opts = self.cfg.to_c()
        need = ctypes.c_size_t()
        N.check("gs_backscatter_workspace_query",
                N.lib().gs_backscatter_workspace_query(ctypes.byref(self.opts), rast.n_views, rast.host_cams,
                                                       ctypes.byref(need)))
        self.workspace = torch.empty(max(need.value, 256), dtype=torch.uint8, device=rast.device)
        nv = rast.n_views
        self.est = torch.zeros(nv, 6, dtype=torch.float32, device=rast.device)
        self.points = torch.empty(nv, 3, self.cfg.intervals - 1, 2, dtype=torch.float32, device=rast.device)
        self.cost = torch.empty(nv, 3, dtype=torch.float32, device=rast.device)

    def __call__(self, image: torch.Tensor, depth: torch.Tensor) -> torch.Tensor:
        """image packed like the rgb output (observed views), depth like the depth output; returns the
        [views, 6] estimates (B_inf_hat[3], B_b_hat[3]); points and cost stay in the attributes."""
        image = _f32(image)
        depth = _f32(depth)
        N.check("gs_estimate_backscatter",
                N.lib().gs_estimate_backscatter(ctypes.byref(self.opts), self.rast.n_views, self.rast.host_cams,
                                                _ptr(image), _ptr(depth), _ptr(self.est), _ptr(self.points),
                                                _ptr(self.cost), _ptr(self.workspace), self.workspace.numel(),
                                                _stream()))
        return self.est


def prior(medium: torch.Tensor, est: torch.Tensor, lam: float,
          grad_medium: Optional[torch.Tensor] = None) -> Tuple[torch.Tensor, Optional[torch.Tensor]]:
    """lam L_best (a [1] tensor) and, when grad_medium is given, lam sign(B - B_hat) added to it."""
    medium = _f32(medium)
    est = _f32(est)
    views = medium.numel() // 9
    loss = torch.empty(1, dtype=torch.float32, device=medium.device)
    N.check("gs_backscatter_prior", N.lib().gs_backscatter_prior(views, _ptr(medium), _ptr(est), float(lam),
                                                                 _ptr(loss), _ptr(grad_medium), _stream()))
    return loss, grad_medium
