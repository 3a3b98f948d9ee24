"""C-ABI checks that need no GPU: the built library loads, exports every
function the header declares, its structs have the header's layout, and the
calls that touch no device behave as documented."""
import ctypes as C
import re
import subprocess
from pathlib import Path

import pytest

from paper_1309_1114_amd import splotch

ROOT = Path(__file__).resolve().parent.parent
HEADER = ROOT / "include" / "splotch.h"
HEADERS = sorted((ROOT / "include").glob("*.h"))


def _no_gpu_process():
    """The checks below start compilers and nm; a process that has already
    initialised a GPU must not start other programs, so they skip there
    (they run in the CPU suite)."""
    try:
        import torch
        if torch.cuda.is_initialized():
            pytest.skip("subprocesses are not started from a GPU-initialised process")
    except ImportError:
        pass


def declared_functions():
    names = set()
    for h in HEADERS:
        text = re.sub(r"/\*.*?\*/", "", h.read_text(), flags=re.S)
        names |= set(re.findall(r"\b(splotch_[a-z_0-9]+)\s*\(", text))
    return sorted(names)


def test_header_declares_the_api():
    names = declared_functions()
    for must in ("splotch_render", "splotch_render_workspace_size", "splotch_ctx_create",
                 "splotch_ctx_destroy", "splotch_get_stats", "splotch_default_params",
                 "splotch_nn_conv3x3_fwd", "splotch_nn_conv3x3_bwd_weight", "splotch_nn_head",
                 "splotch_nn_adam", "splotch_nn_consistency"):
        assert must in names


def test_library_exports_every_declared_symbol():
    _no_gpu_process()
    lib = splotch.load()
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    out = subprocess.run(["nm", "-D", "--defined-only", str(splotch.LIB_PATH)],
                         capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\bT (splotch_\w+)", out))
    assert set(declared_functions()) <= exported


LAYOUT_C = r"""
#include <stdio.h>
#include <stddef.h>
#include "splotch.h"
#define S(t) printf(#t " %zu\n", sizeof(t));
#define O(t, f) printf(#t "." #f " %zu\n", offsetof(t, f));
int main(void) {
  S(splotch_particles) O(splotch_particles, species) O(splotch_particles, vz)
  S(splotch_camera) O(splotch_camera, fov_deg) O(splotch_camera, height)
  S(splotch_colormap) O(splotch_colormap, rgb)
  S(splotch_params) O(splotch_params, scalar_min) O(splotch_params, accum) O(splotch_params, chunk)
  O(splotch_params, colour_mode) O(splotch_params, transfer) O(splotch_params, absorption)
  S(splotch_image) O(splotch_image, center_count)
  S(splotch_stats) O(splotch_stats, overflow) O(splotch_stats, chunk)
  O(splotch_stats, radius_hist) O(splotch_stats, radius_mean) O(splotch_stats, n_samples)
  return 0;
}
"""


def test_struct_layout_matches_ctypes(tmp_path):
    _no_gpu_process()
    src = tmp_path / "layout.c"
    src.write_text(LAYOUT_C)
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", f"-I{ROOT / 'include'}", str(src), "-o", str(exe)],
                   check=True)
    got = dict(line.rsplit(" ", 1) for line in
               subprocess.run([str(exe)], capture_output=True, text=True).stdout.splitlines())
    py = {
        "splotch_particles": splotch.Particles, "splotch_camera": splotch.CameraS,
        "splotch_colormap": splotch.Colormap, "splotch_params": splotch.ParamsS,
        "splotch_image": splotch.Image, "splotch_stats": splotch.Stats,
    }
    for key, val in got.items():
        if "." in key:
            t, f = key.split(".")
            assert getattr(py[t], f).offset == int(val), key
        else:
            assert C.sizeof(py[key]) == int(val), key


def test_host_only_calls():
    lib = splotch.load()
    assert lib.splotch_abi_version() == 7
    assert lib.splotch_status_string(0) == b"SPLOTCH_OK"
    assert lib.splotch_status_string(-2) == b"SPLOTCH_ERR_WORKSPACE"
    p = splotch.ParamsS()
    assert lib.splotch_default_params(C.byref(p)) == 0
    assert p.chi == 3.0 and p.frac_bits == 40 and p.halo == -1 and p.accum == 0
    assert p.colour_mode == 0 and p.transfer == 0 and list(p.absorption) == [0.0] * 4
    assert list(p.brightness) == [1.0] * 4
    assert lib.splotch_default_params(None) == splotch.ERR_INVALID_ARG
    # NULL context / NULL outputs are rejected before touching a device
    assert lib.splotch_render(None, None, None, None, None, None, None, 0, None) == -1
    assert lib.splotch_render_workspace_size(None, None, None, None, None) == -1
    assert lib.splotch_get_stats(None, None, None) == -1
    assert lib.splotch_ctx_create(None, 0) == -1
    assert lib.splotch_ctx_destroy(None) == 0
    assert lib.splotch_last_error(None) == b"no context"


def test_nn_argument_errors_need_no_device():
    lib = splotch.load()
    f = lib.splotch_nn_conv3x3_fwd
    f.restype = C.c_int32
    f.argtypes = [C.c_void_p] * 5 + [C.c_int32] * 7 + [C.c_void_p]
    fake = C.c_void_p(1 << 20)
    assert f(None, fake, None, None, fake, 1, 8, 8, 32, 32, 1, 0, None) == splotch.ERR_INVALID_ARG
    assert f(fake, fake, None, None, fake, 1, 8, 8, 32, 40, 1, 0, None) == splotch.ERR_UNSUPPORTED
    assert f(fake, fake, None, None, fake, 1, 8, 8, 48, 48, 1, 0, None) == splotch.ERR_UNSUPPORTED
    assert f(fake, fake, None, None, fake, 0, 8, 8, 32, 32, 1, 0, None) == splotch.ERR_INVALID_ARG
    g = lib.splotch_nn_conv3x3_bwd_weight
    g.restype = C.c_int32
    g.argtypes = [C.c_void_p] * 5 + [C.c_int32] * 5 + [C.c_void_p]
    assert g(fake, fake, None, fake, None, 1, 8, 8, 48, 32, None) == splotch.ERR_UNSUPPORTED
    a = lib.splotch_nn_adam
    a.restype = C.c_int32
    a.argtypes = [C.c_void_p] * 4 + [C.c_int64] + [C.c_float] * 4 + [C.c_int32, C.c_void_p]
    assert a(fake, fake, fake, fake, 10, 1e-3, 0.9, 0.999, 1e-8, 0, None) == splotch.ERR_INVALID_ARG
    assert a(fake, fake, fake, fake, 0, 1e-3, 0.9, 0.999, 1e-8, 1, None) == splotch.OK
