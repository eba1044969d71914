"""The allocation-free loss entry point (gs_l1_dssim_loss_noalloc) against gs_l1_dssim_loss, both
called through the C ABI: two calls in a row on one GPU, the second with fewer and smaller views,
so the library's fixed scratch array holds the first call's partial sums when the second starts."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2411_19588_amd import _native as N
from paper_2411_19588_amd import synth

pytestmark = pytest.mark.gpu


def _cams(sizes):
    return N.camera_array([synth.Camera(w, h, float(w), float(w), w / 2.0, h / 2.0, np.eye(3, dtype=np.float32),
                                        np.zeros(3, np.float32)) for w, h in sizes])


def _pair(sizes, seed):
    rng = np.random.default_rng(seed)
    n = sum(3 * w * h for w, h in sizes)
    tgt = rng.uniform(size=n).astype(np.float32)
    pred = np.clip(tgt + rng.normal(0, 0.1, size=n), 0, 1).astype(np.float32)
    return torch.from_numpy(pred).cuda(), torch.from_numpy(tgt).cuda()


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _with_workspace(L, cams, nv, pred, tgt, lam, stream):
    need = ctypes.c_size_t()
    N.check("gs_loss_workspace_query", L.gs_loss_workspace_query(nv, cams, ctypes.byref(need)))
    ws = torch.empty(max(need.value, 256), dtype=torch.uint8, device="cuda")
    loss = torch.empty(nv + 1, dtype=torch.float32, device="cuda")
    grad = torch.empty_like(pred)
    N.check("gs_l1_dssim_loss", L.gs_l1_dssim_loss(nv, cams, _ptr(pred), _ptr(tgt), lam, _ptr(loss), _ptr(grad),
                                                   _ptr(ws), ws.numel(), stream))
    return loss, grad


def _no_alloc(L, cams, nv, pred, tgt, lam, stream):
    loss = torch.empty(nv + 1, dtype=torch.float32, device="cuda")
    grad = torch.empty_like(pred)
    N.check("gs_l1_dssim_loss_noalloc", L.gs_l1_dssim_loss_noalloc(nv, cams, _ptr(pred), _ptr(tgt), lam, _ptr(loss),
                                                                   _ptr(grad), stream))
    return loss, grad


def test_no_alloc_loss_matches_workspace_entry_point():
    L = N.lib()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    lam = ctypes.c_float(0.3)
    calls = [[(1920, 1080), (640, 480), (203, 141)], [(97, 61)]]
    for i, sizes in enumerate(calls):
        cams = _cams(sizes)
        pred, tgt = _pair(sizes, 7 + i)
        # the allocation-free call first, so its partial sums cannot come from the other call
        loss_n, grad_n = _no_alloc(L, cams, len(sizes), pred, tgt, lam, stream)
        torch.cuda.synchronize()
        loss_w, grad_w = _with_workspace(L, cams, len(sizes), pred, tgt, lam, stream)
        torch.cuda.synchronize()
        # same kernels, same fixed-order reductions: bit-identical results
        assert torch.equal(loss_n, loss_w), (i, loss_n.cpu().numpy(), loss_w.cpu().numpy())
        assert torch.equal(grad_n, grad_w), i
        assert np.isfinite(loss_n.cpu().numpy()).all()
        print(f"call {i}: {len(sizes)} views, loss {loss_n[-1].item():.6f}", flush=True)


def test_no_alloc_rejects_too_many_workgroups():
    L = N.lib()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    sizes = [(4096, 4096)] * 11   # 3 * 128 * 256 * 11 = 1,081,344 workgroups > 2^20
    cams = _cams(sizes)
    x = torch.zeros(16, dtype=torch.float32, device="cuda")
    rc = L.gs_l1_dssim_loss_noalloc(len(sizes), cams, _ptr(x), _ptr(x), ctypes.c_float(0.3), _ptr(x), _ptr(x), stream)
    assert rc == N.GS_ERR_WORKSPACE_TOO_SMALL
