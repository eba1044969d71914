"""The C-ABI library loads and exports every declared symbol; host-only calls and
argument validation work without a GPU (no compute call is made here)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2411_19588_amd import _native as N
from paper_2411_19588_amd import synth

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "gsplash.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(gs_[a-z0-9_]+)\s*\(", src)
    return sorted(set(names))


def test_every_declared_symbol_is_exported_and_bound():
    L = N.lib()
    names = declared_functions()
    assert len(names) >= 15
    for name in names:
        assert hasattr(L, name), name
        assert name in N.PROTOTYPES, f"{name} has no ctypes prototype"


def test_struct_layouts_match_header(tmp_path):
    """sizeof/offsetof of every ABI struct, as a C compiler sees the header, equal the ctypes mirrors."""
    structs = {"gs_camera": N.GsCamera, "gs_gaussians": N.GsGaussians, "gs_gaussian_grads": N.GsGaussianGrads,
               "gs_options": N.GsOptions, "gs_adam_group": N.GsAdamGroup,
               "gs_backscatter_options": N.GsBackscatterOptions, "gs_mcmc_state": N.GsMcmcState}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "gsplash.h"', "int main(void) {"]
    for cname, cls in structs.items():
        lines.append(f'printf("{cname} %zu\\n", sizeof({cname}));')
        for fname, _ in cls._fields_:
            lines.append(f'printf("{cname}.{fname} %zu\\n", offsetof({cname}, {fname}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    import subprocess
    subprocess.check_call(["gcc", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)])
    out = dict(l.rsplit(" ", 1) for l in subprocess.check_output([str(exe)], text=True).splitlines())
    for cname, cls in structs.items():
        assert int(out[cname]) == ctypes.sizeof(cls), cname
        for fname, _ in cls._fields_:
            assert int(out[f"{cname}.{fname}"]) == getattr(cls, fname).offset, (cname, fname)


def test_default_options_and_version():
    o = N.default_options()
    assert (o.tile_w, o.tile_h, o.lds_batch) == (16, 16, 64)
    assert o.alpha_min == pytest.approx(1 / 255) and o.alpha_max == pytest.approx(0.99)
    assert o.t_min == pytest.approx(1e-4) and o.kappa == pytest.approx(11.1)
    assert o.medium_prior is None and o.prior_lambda == 0 and o.reg_opacity == 0 and o.reg_scale == 0
    assert o.phase_limit == 0
    b = N.GsBackscatterOptions()
    N.lib().gs_default_backscatter_options(ctypes.byref(b))
    assert (b.edges, b.intervals, b.resize_height) == (10, 25, 300) and b.p_dark == pytest.approx(0.01)
    assert b"gfx950" in N.lib().gs_version()


def test_schedule_automatic_and_explicit():
    """phases / phase0_shift = 0 resolve automatically: one view bins first the nearest ~1 Gaussian
    per tile (shift = log2 of Gaussians per tile, rounded, clamped to 2..12) in 2 phases; several
    views use 4 phases from the nearest 1/64.  Explicit values pass through; out-of-range ones are
    rejected."""
    sc = synth.make_scene(3, n=10, n_views=3, view_sizes=[(96, 64), (130, 77), (64, 64)])
    cams = N.camera_array(sc.cameras)
    o = N.default_options()
    assert (o.phases, o.phase0_shift) == (0, 0)
    p, sh = ctypes.c_int32(), ctypes.c_int32()

    def sched(n, views):
        assert N.lib().gs_schedule(ctypes.byref(o), n, views, cams, ctypes.byref(p), ctypes.byref(sh)) == 0
        return p.value, sh.value

    tiles = 6 * 4   # the first view, 96x64 in 16x16 tiles
    assert sched(tiles * 128, 1) == (2, 7)
    assert sched(tiles * 45, 1) == (2, 5)          # log2(45) = 5.49
    assert sched(tiles * 46, 1) == (2, 6)          # log2(46) = 5.52
    assert sched(0, 1) == (2, 2) and sched(10, 1) == (2, 2)
    assert sched(tiles << 20, 1) == (2, 12)
    assert sched(10, 3) == (4, 6) and sched(1 << 24, 3) == (4, 6)
    assert N.lib().gs_schedule(ctypes.byref(o), 100, 1, cams, None, None) == 0
    o.phases, o.phase0_shift = 3, 5
    assert sched(tiles * 128, 1) == (3, 5) and sched(10, 3) == (3, 5)
    o.phases = 9
    assert N.lib().gs_schedule(ctypes.byref(o), 10, 3, cams, ctypes.byref(p), ctypes.byref(sh)) == \
        N.GS_ERR_INVALID_ARGUMENT
    o.phases, o.phase0_shift = 0, 0
    assert N.lib().gs_schedule(ctypes.byref(o), -1, 1, cams, ctypes.byref(p), ctypes.byref(sh)) == \
        N.GS_ERR_INVALID_ARGUMENT


def test_workspace_query_and_tile_count():
    sc = synth.make_scene(3, n=1000, n_views=3, view_sizes=[(96, 64), (130, 77), (64, 64)])
    cams = N.camera_array(sc.cameras)
    o = N.default_options()
    ws, sv = ctypes.c_size_t(), ctypes.c_size_t()
    assert N.lib().gs_workspace_query(ctypes.byref(o), 1000, 3, cams, ctypes.byref(ws), ctypes.byref(sv)) == 0
    assert ws.value > o.max_pairs * 16 and sv.value > o.max_pairs * 4   # sort scratch vs stored pair values
    tiles = N.lib().gs_tile_count(ctypes.byref(o), 3, cams)
    assert tiles == 6 * 4 + 9 * 5 + 4 * 4
    o.tile_w = o.tile_h = 8
    o.lds_batch = 64
    assert N.lib().gs_tile_count(ctypes.byref(o), 3, cams) == 12 * 8 + 17 * 10 + 8 * 8
    o.pixels_per_lane = 2                                   # 8x8 tiles take one pixel per lane only
    assert N.lib().gs_workspace_query(ctypes.byref(o), 1000, 3, cams, ctypes.byref(ws), ctypes.byref(sv)) == \
        N.GS_ERR_INVALID_ARGUMENT


@pytest.mark.parametrize("field,value,code", [
    ("tile_w", 12, N.GS_ERR_INVALID_ARGUMENT), ("tile_w", 32, N.GS_ERR_UNSUPPORTED),
    ("lds_batch", 100, N.GS_ERR_INVALID_ARGUMENT), ("alpha_max", 1.5, N.GS_ERR_INVALID_ARGUMENT),
    ("depth_mode", 3, N.GS_ERR_INVALID_ARGUMENT), ("max_pairs", -1, N.GS_ERR_INVALID_ARGUMENT),
    ("max_pairs", 5_000_000_000, N.GS_ERR_INVALID_ARGUMENT), ("pixels_per_lane", 3, N.GS_ERR_INVALID_ARGUMENT),
    ("pixels_per_lane", 8, N.GS_ERR_INVALID_ARGUMENT), ("record_fetch", 3, N.GS_ERR_INVALID_ARGUMENT),
    ("record_fetch", -1, N.GS_ERR_INVALID_ARGUMENT), ("phase0_shift", 21, N.GS_ERR_INVALID_ARGUMENT),
    ("phase0_shift", -1, N.GS_ERR_INVALID_ARGUMENT), ("tile_cull", 2, N.GS_ERR_INVALID_ARGUMENT),
    ("phases", 9, N.GS_ERR_INVALID_ARGUMENT), ("phases", -1, N.GS_ERR_INVALID_ARGUMENT),
    ("depth_output", 2, N.GS_ERR_INVALID_ARGUMENT), ("depth_output", -1, N.GS_ERR_INVALID_ARGUMENT),
    ("phase_limit", 9, N.GS_ERR_INVALID_ARGUMENT), ("phase_limit", -1, N.GS_ERR_INVALID_ARGUMENT)])
def test_bad_options_rejected(field, value, code):
    sc = synth.make_scene(0, n=10)
    cams = N.camera_array(sc.cameras)
    o = N.default_options()
    setattr(o, field, value)
    ws, sv = ctypes.c_size_t(), ctypes.c_size_t()
    assert N.lib().gs_workspace_query(ctypes.byref(o), 10, 1, cams, ctypes.byref(ws), ctypes.byref(sv)) == code


def test_bad_arguments_rejected_before_any_device_work():
    L = N.lib()
    sc = synth.make_scene(0, n=10)
    cams = N.camera_array(sc.cameras)
    o = N.default_options()
    g = N.GsGaussians(10, 0, 0, None, None, None, None, None)     # null parameter arrays
    rc = L.gs_render_forward(ctypes.byref(o), ctypes.byref(g), 1, cams, None, None, None, None, None, None, None,
                             0, None, 0, None)
    assert rc == N.GS_ERR_INVALID_ARGUMENT
    g = N.GsGaussians(10, 4, 0, 1, 1, 1, 1, 1)                     # SH degree 4
    rc = L.gs_render_forward(ctypes.byref(o), ctypes.byref(g), 1, cams, 1, 1, 1, 1, 1, None, 1, 1 << 40, 1, 1 << 40,
                             None)
    assert rc == N.GS_ERR_INVALID_ARGUMENT
    g = N.GsGaussians(10, 0, 0, 1, 1, 1, 1, 1)
    rc = L.gs_render_forward(ctypes.byref(o), ctypes.byref(g), 1, cams, 1, 1, 1, 1, 1, None, 1, 16, 1, 16, None)
    assert rc == N.GS_ERR_WORKSPACE_TOO_SMALL
    rc = L.gs_render_forward(ctypes.byref(o), ctypes.byref(g), 0, cams, 1, 1, 1, 1, 1, None, 1, 16, 1, 16, None)
    assert rc == N.GS_ERR_INVALID_ARGUMENT
    assert L.gs_read_status(None, None, None, None) == N.GS_ERR_INVALID_ARGUMENT
    k = ctypes.c_int32()
    assert L.gs_phases_needed(ctypes.byref(o), 10, 1, cams, None, 1 << 40, ctypes.byref(k), None) == \
        N.GS_ERR_INVALID_ARGUMENT
    assert L.gs_phases_needed(ctypes.byref(o), 10, 1, cams, 1, 16, ctypes.byref(k), None) == \
        N.GS_ERR_WORKSPACE_TOO_SMALL
    assert L.gs_phases_needed(ctypes.byref(o), 10, 1, cams, 1, 1 << 40, None, None) == N.GS_ERR_INVALID_ARGUMENT
    assert L.gs_activate(-1, None, None, None, None, None) == N.GS_ERR_INVALID_ARGUMENT
    assert L.gs_activation(5, 3, 1, 1, None) == N.GS_ERR_INVALID_ARGUMENT
    assert L.gs_activation(5, 1, None, 1, None) == N.GS_ERR_INVALID_ARGUMENT
    assert L.gs_activation(0, 1, None, None, None) == N.GS_OK
    assert L.gs_adam_step_device((N.GsAdamGroup * 1)(), 1, 0.9, 0.999, 1e-8, None, None, None) == \
        N.GS_ERR_INVALID_ARGUMENT
    assert L.gs_l1_loss(0, None, None, None, None, None) == N.GS_ERR_INVALID_ARGUMENT
    grp = (N.GsAdamGroup * 1)()
    grp[0].count = 5
    assert L.gs_adam_step(grp, 1, 0.9, 0.999, 1e-8, 1, None) == N.GS_ERR_INVALID_ARGUMENT
    assert L.gs_adam_step(grp, 1, 0.9, 0.999, 1e-8, 0, None) == N.GS_ERR_INVALID_ARGUMENT
    assert L.gs_adam_step(grp, 9, 0.9, 0.999, 1e-8, 1, None) == N.GS_ERR_INVALID_ARGUMENT


def test_view_limit():
    cams = N.camera_array([synth.make_scene(0, n=1).cameras[0]] * (N.GS_MAX_VIEWS + 1))
    o = N.default_options()
    assert N.lib().gs_tile_count(ctypes.byref(o), N.GS_MAX_VIEWS + 1, cams) == -1


def test_fused_backward_adam_rejects_mismatched_groups():
    """gs_render_backward_adam validates its six groups before any device work."""
    L = N.lib()
    sc = synth.make_scene(0, n=10)
    cams = N.camera_array(sc.cameras)
    o = N.default_options()
    n = 10
    g = N.GsGaussians(n, 0, 0, 0x1000, 0x2000, 0x3000, 0x4000, 0x5000)
    counts = [3 * n, 3 * n, 4 * n, n, 3 * n, 9]
    acts = [0, 1, 0, 2, 0, 0]
    params = [0x1000, 0x6000, 0x3000, 0x7000, 0x5000, 0x8000]
    activated = [0, 0x2000, 0, 0x4000, 0, 0]

    def groups(**change):
        arr = (N.GsAdamGroup * 6)()
        for k in range(6):
            arr[k] = N.GsAdamGroup(params[k], 0x9000, 0xA000, 0xB000, activated[k] or None, counts[k], 1e-3, acts[k], 0)
        for k, (field, value) in change.items():
            setattr(arr[int(k[1:])], field, value)
        return arr

    def call(arr, medium=0x8000):
        return L.gs_render_backward_adam(ctypes.byref(o), ctypes.byref(g), 1, cams, 0xC000, medium, 0xD000, None,
                                         None, 0xE000, 1 << 40, arr, 0.9, 0.999, 1e-8, 0xF000, 0x10000, 1 << 40,
                                         None)

    bad = [dict(g0=("count", 3 * n + 1)), dict(g1=("activation", 0)), dict(g3=("activated", 0x4004)),
           dict(g4=("param", 0x5004)), dict(g5=("grad", None)), dict(g2=("m", None))]
    for change in bad:
        assert call(groups(**change)) == N.GS_ERR_INVALID_ARGUMENT, change
    assert call(groups(), medium=0x8004) == N.GS_ERR_INVALID_ARGUMENT


def test_backscatter_argument_checks():
    """Host-only validation of the backscatter entry points (nothing is enqueued on error)."""
    L = N.lib()
    cams = N.camera_array([synth.Camera(w, h, float(w), float(w), w / 2, h / 2, np.eye(3, dtype=np.float32),
                                        np.zeros(3, np.float32)) for w, h in ((1920, 1080), (640, 480))])
    o = N.GsBackscatterOptions()
    L.gs_default_backscatter_options(ctypes.byref(o))
    need = ctypes.c_size_t()
    assert L.gs_backscatter_workspace_query(ctypes.byref(o), 2, cams, ctypes.byref(need)) == N.GS_OK
    # 533 x 300 + 400 x 300 resized pixels: image, depth, segment, 4 sort buffers
    assert need.value >= (533 * 300 + 400 * 300) * 9 * 4
    for field, bad in (("edges", 1), ("edges", 34), ("intervals", 1), ("intervals", 258), ("p_dark", 0.0),
                       ("p_dark", 1.5), ("resize_height", -1)):
        b = N.GsBackscatterOptions.from_buffer_copy(o)
        setattr(b, field, bad)
        assert L.gs_backscatter_workspace_query(ctypes.byref(b), 2, cams, ctypes.byref(need)) == \
            N.GS_ERR_INVALID_ARGUMENT, field
    assert L.gs_backscatter_workspace_query(ctypes.byref(o), 0, cams, ctypes.byref(need)) == N.GS_ERR_INVALID_ARGUMENT
    p = ctypes.c_void_p(16)
    assert L.gs_estimate_backscatter(ctypes.byref(o), 2, cams, None, p, p, None, None, p, 1 << 30, None) == \
        N.GS_ERR_INVALID_ARGUMENT
    assert L.gs_estimate_backscatter(ctypes.byref(o), 2, cams, p, p, p, None, None, p, 16, None) == \
        N.GS_ERR_WORKSPACE_TOO_SMALL
    assert L.gs_backscatter_prior(0, p, p, 0.1, p, p, None) == N.GS_ERR_INVALID_ARGUMENT
    assert L.gs_backscatter_prior(2, p, p, -1.0, p, p, None) == N.GS_ERR_INVALID_ARGUMENT
    assert L.gs_backscatter_prior(2, p, p, 0.1, None, None, None) == N.GS_ERR_INVALID_ARGUMENT


def test_mcmc_add_count_and_argument_checks():
    """gs_mcmc_add_count (host) against the oracle's count; MCMC entry points reject bad arguments
    before any device work."""
    from oracle import mcmc as M
    L = N.lib()
    for n, cap in ((1000, 5000), (1000, 1030), (1000, 1000), (1000, 900), (3_000_000, 3_100_000), (19, 100), (1, 10)):
        assert L.gs_mcmc_add_count(n, cap, ctypes.c_double(1.05)) == M.add_count(n, cap), (n, cap)
    need = ctypes.c_size_t()
    assert L.gs_mcmc_workspace_query(1000, 1000, ctypes.byref(need)) == N.GS_OK and need.value >= 1000 * 20
    assert L.gs_mcmc_workspace_query(0, 10, ctypes.byref(need)) == N.GS_ERR_INVALID_ARGUMENT
    st = N.GsMcmcState()
    st.n = 100
    st.sh_degree = 1
    p = 4096
    for k in range(5):
        st.param[k] = st.m[k] = st.v[k] = p
    st.scales = st.opacity = p
    d = ctypes.c_void_p(p)
    assert L.gs_mcmc_relocate(ctypes.byref(st), 0.1, None, None, None, d, 1 << 30, None) == N.GS_ERR_INVALID_ARGUMENT
    assert L.gs_mcmc_relocate(ctypes.byref(st), 1.5, d, None, None, d, 1 << 30, None) == N.GS_ERR_INVALID_ARGUMENT
    assert L.gs_mcmc_relocate(ctypes.byref(st), 0.1, d, None, None, d, 16, None) == N.GS_ERR_WORKSPACE_TOO_SMALL
    bad = N.GsMcmcState.from_buffer_copy(st)
    bad.sh_degree = 4
    assert L.gs_mcmc_relocate(ctypes.byref(bad), 0.1, d, None, None, d, 1 << 30, None) == N.GS_ERR_INVALID_ARGUMENT
    small = N.GsMcmcState.from_buffer_copy(st)
    small.n = 50
    assert L.gs_mcmc_add(ctypes.byref(st), ctypes.byref(small), d, None, None, d, 1 << 30, None) == \
        N.GS_ERR_INVALID_ARGUMENT
    assert L.gs_mcmc_noise(-1, d, d, d, d, d, 1.0, 1.0, None) == N.GS_ERR_INVALID_ARGUMENT
