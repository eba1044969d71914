"""Fused Adam over the Gaussian and medium parameters (gs_adam_step).

Sec. Optimization trains every parameter with Adam at the 3DGS learning rates
and the medium coefficients at the colour learning rate.  Scales and
opacities are stored raw (log-scale, logit); the kernel takes gradients
w.r.t. the activated values, chains them through exp / sigmoid, updates the
raw values and writes the new activated values in the same pass.
"""
from __future__ import annotations

import ctypes
import dataclasses
from typing import List, Optional

import torch

from . import _native as N

# Learning rates of the appendix "Experimental Setup" (position: initial value).
LR = dict(means=0.00016, sh=0.0025, medium=0.0025, opacity=0.05, scales=0.005, quats=0.001)

_ACT = {None: 0, "exp": 1, "sigmoid": 2}


@dataclasses.dataclass
class Group:
    name: str
    param: torch.Tensor
    lr: float
    activation: Optional[str] = None
    grad: Optional[torch.Tensor] = None
    m: Optional[torch.Tensor] = None
    v: Optional[torch.Tensor] = None
    activated: Optional[torch.Tensor] = None

    def __post_init__(self):
        if self.param.dtype != torch.float32 or not self.param.is_contiguous():
            raise ValueError("parameters must be contiguous float32")
        if self.activation not in _ACT:
            raise ValueError(f"unknown activation {self.activation}")
        z = lambda: torch.zeros_like(self.param)
        self.grad = z() if self.grad is None else self.grad
        self.m = z() if self.m is None else self.m
        self.v = z() if self.v is None else self.v
        if self.activation and self.activated is None:
            # one-time set-up of the activated copy (gs_activation); every step refreshes it in the kernel
            self.activated = torch.empty_like(self.param)
            s = torch.cuda.current_stream(self.param.device)
            N.check("gs_activation", N.lib().gs_activation(self.param.numel(), _ACT[self.activation],
                                                           ctypes.c_void_p(self.param.data_ptr()),
                                                           ctypes.c_void_p(self.activated.data_ptr()),
                                                           ctypes.c_void_p(s.cuda_stream)))


class FusedAdam:
    def __init__(self, groups: List[Group], betas=(0.9, 0.999), eps=1e-8):
        if not 1 <= len(groups) <= 8:
            raise ValueError("1..8 parameter groups per launch")
        self.groups = groups
        self.betas = betas
        self.eps = eps
        self.step_count = 0

    def group(self, name: str) -> Group:
        for g in self.groups:
            if g.name == name:
                return g
        raise KeyError(name)

    def step(self, stream=None) -> None:
        self.step_count += 1
        arr = (N.GsAdamGroup * len(self.groups))()
        for i, g in enumerate(self.groups):
            arr[i] = N.GsAdamGroup(g.param.data_ptr(), g.grad.data_ptr(), g.m.data_ptr(), g.v.data_ptr(),
                                   g.activated.data_ptr() if g.activated is not None else None,
                                   g.param.numel(), g.lr, _ACT[g.activation], 0)
        s = torch.cuda.current_stream() if stream is None else stream
        N.check("gs_adam_step", N.lib().gs_adam_step(arr, len(self.groups), self.betas[0], self.betas[1], self.eps,
                                                     self.step_count, ctypes.c_void_p(s.cuda_stream)))
