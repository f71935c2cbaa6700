"""The C ABI library: it loads, exports every entry point that include/fbpnp.h declares,
and rejects invalid arguments on the host before any launch (no GPU needed)."""
import ctypes
import math
import os
import re

import pytest

from paper_2203_07308_amd import fbpnp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "fbpnp.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return re.findall(r"^\s*(?:fb_status|size_t|int32_t|const char\*)\s+(\w+)\s*\(", text, flags=re.M)


def test_library_exports_every_declared_symbol():
    lib = fbpnp.load()
    names = header_functions()
    assert len(names) >= 15
    assert sorted(names) == sorted(fbpnp.EXPORTS)
    for n in names:
        assert hasattr(lib, n), n


def geom(**kw):
    base = dict(nx=64, ny=64, pixel_mm=1.0, n_views=90, n_bins=96, sod_mm=500.0, sdd_mm=1000.0, det_pitch_mm=2.0)
    base.update(kw)
    return fbpnp.Geometry(**base)


def create(g, factors):
    lib = fbpnp.load()
    arr = (ctypes.c_int32 * len(factors))(*factors)
    h = ctypes.c_void_p()
    st = lib.fb_plan_create(ctypes.byref(g.c()), len(factors), arr, ctypes.byref(h))
    return st, lib.fb_last_error().decode(), h


@pytest.mark.parametrize("kw,code", [
    (dict(sod_mm=40.0), -2),                 # source inside the image circumcircle
    (dict(sdd_mm=90.0), -2),                 # fan wider than 90 degrees
    (dict(pixel_mm=float("nan")), -2),       # non-finite
    (dict(det_pitch_mm=0.0), -2),
    (dict(nx=0), -1),
    (dict(n_views=0), -1),
])
def test_plan_rejects_bad_geometry(kw, code):
    st, msg, h = create(geom(**kw), [1])
    assert st == code and msg and not h.value


def test_plan_rejects_bad_factors():
    assert create(geom(), [3])[0] == -3
    assert create(geom(), [1, 0])[0] == -1
    assert create(geom(nx=64, ny=48), [1, 32])[0] == -3


def test_calls_reject_bad_arguments():
    lib = fbpnp.load()
    p = ctypes.c_void_p(16)
    assert lib.fanbeam_fp(None, 0, p, p, None, 90, None) == -1
    assert "plan" in lib.fb_last_error().decode()
    assert lib.fanbeam_bp(None, 0, p, p, None, 90, ctypes.c_float(1.0), None) == -1
    assert lib.sketch_down(p, 9, 8, 2, p, None) == -3
    assert lib.sketch_down(None, 8, 8, 2, p, None) == -1
    assert lib.sketch_up(p, 4, 4, 0, p, None) == -1
    assert lib.tv_prox(p, p, 8, 8, ctypes.c_float(0.01), 5, ctypes.c_float(0.125), None, 0, None) == -1  # alias
    q = ctypes.c_void_p(32)
    assert lib.tv_prox(p, q, 8, 8, ctypes.c_float(-1.0), 5, ctypes.c_float(0.125), None, 0, None) == -1
    assert lib.tv_prox(p, q, 8, 8, ctypes.c_float(0.01), 50, ctypes.c_float(0.125), None, 0, None) == -1  # no ws
    assert lib.pnp_step(None, None, None) == -1
    assert lib.fb_graph_create(None, None, 0, None) == -1
    assert lib.fb_graph_launch(None, None) == -1
    assert lib.fb_power_lipschitz(None, 0, 10, None, None) == -1
    assert lib.fb_plan_destroy(None) == 0
    assert lib.fb_graph_destroy(None) == 0


def test_tv_workspace_size():
    lib = fbpnp.load()
    assert lib.fb_tv_workspace_bytes(64, 32, 5) == 0
    assert lib.fb_tv_workspace_bytes(64, 32, 8) == 0
    assert lib.fb_tv_workspace_bytes(64, 32, 9) == 4 * 64 * 32 * 4


def test_tv_vjp_workspace_size():
    """Up to 5 denoiser steps the reverse sweep runs in one launch with no workspace."""
    lib = fbpnp.load()
    for k in range(6):
        assert lib.fb_tv_vjp_workspace_bytes(64, 32, k) == 0
    # p levels 0..K (two planes each), u levels 0..K-1, pbar and qbar (two planes each)
    assert lib.fb_tv_vjp_workspace_bytes(64, 32, 6) == 4 * 64 * 32 * (2 * 7 + 6 + 4)
    assert lib.fb_tv_vjp_workspace_bytes(0, 32, 6) == 0


def test_struct_layouts_match_header(tmp_path):
    """ctypes mirrors agree with the C compiler's layout of the header's structs."""
    import shutil
    import subprocess

    if shutil.which("gcc") is None or not os.path.isdir("/opt/rocm/include"):
        pytest.skip("needs gcc and the ROCm headers")
    src = tmp_path / "layout.c"
    src.write_text("""
#include <stdio.h>
#include <stddef.h>
#include "fbpnp.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu %zu\\n", sizeof(fb_geom), offsetof(fb_geom, angle_step_rad),
         sizeof(fb_stage_info), sizeof(fb_pnp_args), offsetof(fb_pnp_args, b),
         offsetof(fb_pnp_args, tv_iters), offsetof(fb_pnp_args, history), offsetof(fb_pnp_args, events));
  printf("%zu %zu %zu %zu\\n", offsetof(fb_pnp_args, vr_mode), offsetof(fb_pnp_args, snap_grad),
         offsetof(fb_pnp_args, grad), offsetof(fb_pnp_args, stamp));
  printf("%zu %zu %zu %zu %zu %zu\\n", sizeof(fb_launch_config), sizeof(fb_batch_args), offsetof(fb_batch_args, eta),
         offsetof(fb_batch_args, tv_iters), offsetof(fb_batch_args, history), offsetof(fb_batch_args, events));
  return 0;
}
""")
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"),
                           "-I", "/opt/rocm/include", str(src), "-o", str(exe)])
    got = [int(v) for v in subprocess.check_output([str(exe)]).split()]
    want = [ctypes.sizeof(fbpnp.Geom), fbpnp.Geom.angle_step_rad.offset, ctypes.sizeof(fbpnp.StageInfo),
            ctypes.sizeof(fbpnp.PnpArgs), fbpnp.PnpArgs.b.offset, fbpnp.PnpArgs.tv_iters.offset,
            fbpnp.PnpArgs.history.offset, fbpnp.PnpArgs.events.offset,
            fbpnp.PnpArgs.vr_mode.offset, fbpnp.PnpArgs.snap_grad.offset, fbpnp.PnpArgs.grad.offset,
            fbpnp.PnpArgs.stamp.offset,
            ctypes.sizeof(fbpnp.LaunchConfig), ctypes.sizeof(fbpnp.BatchArgs), fbpnp.BatchArgs.eta.offset,
            fbpnp.BatchArgs.tv_iters.offset, fbpnp.BatchArgs.history.offset, fbpnp.BatchArgs.events.offset]
    assert got == want
    assert math.isclose(geom().c().angle_step_rad, 2 * math.pi / 90)
