"""PyTorch front end of the MCMC densification kernels (Sec. Implementation; appendix "Experimental
Setup": every 100 iterations, minimum opacity 0.1): relocation of dead Gaussians, addition up to a
capacity, Langevin noise on the means.  Argument marshalling only (gs_mcmc_relocate, gs_mcmc_add,
gs_mcmc_noise do the work); the random numbers the method draws are inputs, taken from a seeded
torch generator on the device (u32 draws, standard normal noise).
"""
from __future__ import annotations

import ctypes
from typing import Dict, Optional, Tuple

import torch

from . import _native as N
from .rasterizer import _ptr, _stream

GROUPS = ("means", "log_scales", "quats", "logits", "sh")
DEAD_OPACITY = 0.1      # appendix "Experimental Setup": minimum opacity threshold
GROWTH = 1.05
NOISE_LR = 5e5


def state_of(t: Dict[str, torch.Tensor], sh_degree: int) -> N.GsMcmcState:
    """t holds, per group g of GROUPS, 'g' (raw parameter planes), 'm_g', 'v_g', and the activated
    copies 'scales' and 'opacity'; every tensor contiguous float32 with n columns."""
    n = int(t["opacity"].numel())
    st = N.GsMcmcState()
    st.n = n
    st.sh_degree = int(sh_degree)
    for k, g in enumerate(GROUPS):
        for key, arr in ((g, st.param), ("m_" + g, st.m), ("v_" + g, st.v)):
            x = t[key]
            if x.dtype != torch.float32 or not x.is_contiguous() or x.shape[-1] != n:
                raise ValueError(f"{key}: contiguous float32 planes of {n} Gaussians expected")
            arr[k] = x.data_ptr()
    st.scales = t["scales"].data_ptr()
    st.opacity = t["opacity"].data_ptr()
    return st


def _workspace(n: int, draws: int, device) -> torch.Tensor:
    need = ctypes.c_size_t()
    N.check("gs_mcmc_workspace_query", N.lib().gs_mcmc_workspace_query(n, draws, ctypes.byref(need)))
    return torch.empty(max(need.value, 256), dtype=torch.uint8, device=device)


def relocate(t: Dict[str, torch.Tensor], sh_degree: int, draws: torch.Tensor,
             dead_opacity: float = DEAD_OPACITY) -> Tuple[torch.Tensor, torch.Tensor]:
    """In place.  draws: int32 [n] (u32 bit patterns).  Returns (sources [n] int32 of which the first
    `taken` are valid, taken [1] int32), both on the device."""
    n = int(t["opacity"].numel())
    dev = t["opacity"].device
    st = state_of(t, sh_degree)
    src = torch.empty(n, dtype=torch.int32, device=dev)
    taken = torch.zeros(1, dtype=torch.int32, device=dev)
    ws = _workspace(n, n, dev)
    N.check("gs_mcmc_relocate", N.lib().gs_mcmc_relocate(ctypes.byref(st), float(dead_opacity), _ptr(draws),
                                                         _ptr(src), _ptr(taken), _ptr(ws), ws.numel(), _stream()))
    return src, taken


def add(t: Dict[str, torch.Tensor], sh_degree: int, capacity: int, draws: torch.Tensor,
        growth: float = GROWTH) -> Tuple[Dict[str, torch.Tensor], torch.Tensor, torch.Tensor]:
    """Out of place.  Returns (new tensors with n + k columns, sources [k], taken [1]); k from
    gs_mcmc_add_count.  When taken is 0 (no Gaussian with a weight) keep the old tensors."""
    n = int(t["opacity"].numel())
    dev = t["opacity"].device
    k = int(N.lib().gs_mcmc_add_count(n, int(capacity), float(growth)))
    out = {key: torch.empty(x.shape[:-1] + (n + k,), dtype=torch.float32, device=dev) for key, x in t.items()}
    a, b = state_of(t, sh_degree), state_of(out, sh_degree)
    src = torch.empty(max(k, 1), dtype=torch.int32, device=dev)
    taken = torch.zeros(1, dtype=torch.int32, device=dev)
    if draws.numel() < k:
        raise ValueError(f"{k} draws needed")
    ws = _workspace(n, k, dev)
    N.check("gs_mcmc_add", N.lib().gs_mcmc_add(ctypes.byref(a), ctypes.byref(b), _ptr(draws), _ptr(src), _ptr(taken),
                                               _ptr(ws), ws.numel(), _stream()))
    return out, src[:k], taken


def noise(means: torch.Tensor, quats: torch.Tensor, scales: torch.Tensor, opacity: torch.Tensor, eta: torch.Tensor,
          lr_means: float, noise_lr: float = NOISE_LR) -> None:
    """In place on means ([3][n]); eta [3][n] standard normal draws."""
    n = int(opacity.numel())
    N.check("gs_mcmc_noise", N.lib().gs_mcmc_noise(n, _ptr(means), _ptr(quats), _ptr(scales), _ptr(opacity),
                                                   _ptr(eta), float(lr_means), float(noise_lr), _stream()))


class Densifier:
    """Seeded source of the method's random numbers and the densification schedule's constants."""

    def __init__(self, device="cuda", seed: int = 0, dead_opacity: float = DEAD_OPACITY, growth: float = GROWTH,
                 noise_lr: float = NOISE_LR):
        self.gen = torch.Generator(device=device)
        self.gen.manual_seed(seed)
        self.device = torch.device(device)
        self.dead_opacity = dead_opacity
        self.growth = growth
        self.noise_lr = noise_lr

    def draws(self, count: int) -> torch.Tensor:
        """count uniform u32 values (as int32 bit patterns)."""
        return torch.randint(-(1 << 31), 1 << 31, (max(count, 1),), dtype=torch.int32, generator=self.gen,
                             device=self.device)

    def normals(self, n: int) -> torch.Tensor:
        return torch.randn((3, n), dtype=torch.float32, generator=self.gen, device=self.device)
