"""The C ABI library loads, exports what its header declares, and validates
arguments on the host (no GPU needed: nothing here launches a kernel)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "speedysplat.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(ss_\w+)\s*\(", text, re.M)))


@pytest.fixture(scope="module")
def L():
    from paper_2412_00578_amd import _lib
    return _lib.lib()


def test_header_declares_the_stages():
    names = declared_functions()
    for n in ("ss_preprocess", "ss_depth_order", "ss_scan", "ss_emit", "ss_sort", "ss_ranges",
              "ss_blend", "ss_render", "ss_forward_begin", "ss_forward_finish",
              "ss_get_constants"):
        assert n in names


def test_every_declared_symbol_is_exported_and_bound(L):
    from paper_2412_00578_amd import _lib
    for name in declared_functions():
        assert hasattr(L, name), name
        assert name in _lib.PROTOTYPES, f"{name} has no ctypes prototype"


def test_constants_match_independent_values(L):
    from paper_2412_00578_amd import _lib
    c = _lib.constants()
    assert c.abi_version == 5 and c.tile == 16
    assert c.alpha_min == pytest.approx(1 / 255, rel=1e-7)
    assert c.alpha_max == pytest.approx(0.99, rel=1e-7)
    assert c.t_min == pytest.approx(1e-4, rel=1e-7)
    assert c.dilation == pytest.approx(0.3, rel=1e-7)
    assert c.fov_clamp == pytest.approx(1.3, rel=1e-7)
    assert c.disc_floor == pytest.approx(0.1, rel=1e-7)


def test_status_strings(L):
    for s in range(5):
        assert L.ss_status_string(s)
    assert L.ss_status_string(99) == b"unknown status"


def test_frame_sizes(L):
    from paper_2412_00578_amd import _lib
    info = _lib.SSFrameInfo()
    assert L.ss_frame_sizes(1_500_000, 1600, 1040, ctypes.byref(info)) == 0
    assert (info.tiles_x, info.tiles_y, info.n_tiles) == (100, 65, 6500)
    assert info.sort_bits == 13
    assert info.scan_tmp_words == 1 + (1_500_000 + 4095) // 4096
    assert L.ss_frame_sizes(10, 1920, 1080, ctypes.byref(info)) == 0
    assert (info.tiles_x, info.tiles_y) == (120, 68)
    assert L.ss_frame_sizes(10, 256, 256, ctypes.byref(info)) == 0 and info.sort_bits == 8
    assert L.ss_frame_sizes(-1, 16, 16, ctypes.byref(info)) == _lib.SS_ERR_INVALID_ARG
    assert L.ss_frame_sizes(1, 0, 16, ctypes.byref(info)) == _lib.SS_ERR_INVALID_ARG


def _cam(**kw):
    from paper_2412_00578_amd import _lib
    c = _lib.SSCamera()
    c.width, c.height = kw.get("w", 64), kw.get("h", 64)
    c.fx = c.fy = kw.get("f", 64.0)
    c.cx, c.cy = 32.0, 32.0
    c.R[0] = c.R[4] = c.R[8] = 1.0
    c.near_z = 0.2
    return c


def test_invalid_arguments_rejected_before_launch(L):
    from paper_2412_00578_amd import _lib
    bad = _lib.SS_ERR_INVALID_ARG
    g = _lib.SSGaussians()
    g.n, g.sh_degree, g.sh_stride = 10, 0, 1  # null parameter pointers
    f = _lib.SSFrame()
    cam = _cam()
    assert L.ss_preprocess(None, ctypes.byref(g), 2, ctypes.byref(f), None) == bad
    assert L.ss_preprocess(ctypes.byref(cam), ctypes.byref(g), 2, ctypes.byref(f), None) == bad
    assert b"NULL" in L.ss_last_error()
    g.n, g.sh_degree = 0, 4
    assert L.ss_preprocess(ctypes.byref(cam), ctypes.byref(g), 2, ctypes.byref(f), None) == bad
    assert b"sh_degree" in L.ss_last_error()
    g.sh_degree = 0
    assert L.ss_preprocess(ctypes.byref(cam), ctypes.byref(g), 7, ctypes.byref(f), None) == bad
    cam0 = _cam(w=0)
    assert L.ss_preprocess(ctypes.byref(cam0), ctypes.byref(g), 2, ctypes.byref(f), None) == bad
    camf = _cam(f=-1.0)
    assert L.ss_preprocess(ctypes.byref(camf), ctypes.byref(g), 2, ctypes.byref(f), None) == bad


def test_records_must_be_interleaved(L):
    # frame.conic must be frame.geom + 4 floats (one [n, 8] record buffer); a
    # frame with separate arrays is rejected before anything is launched
    import numpy as np
    from paper_2412_00578_amd import _lib
    n = 10
    host = np.zeros(1 << 16, dtype=np.uint8)
    base = (host.ctypes.data + 255) // 256 * 256
    g = _lib.SSGaussians()
    g.n, g.sh_degree, g.sh_stride = n, 0, 1
    for k, name in enumerate(("means", "scales", "quats", "opacity", "sh")):
        setattr(g, name, base + 1024 * k)
    f = _lib.SSFrame()
    for k, (name, _) in enumerate(_lib.SSFrame._fields_):
        setattr(f, name, base + 8192 + 1024 * k)
    f.conic = f.geom + 4 * n * 4          # a separate [n, 4] array after geom
    assert L.ss_preprocess(ctypes.byref(_cam()), ctypes.byref(g), 2, ctypes.byref(f),
                           None) == _lib.SS_ERR_INVALID_ARG
    assert b"interleaved" in L.ss_last_error()


def test_workspace_and_overflow_checks(L):
    from paper_2412_00578_amd import _lib
    p = _lib.SSPairs()
    p.capacity = 100
    f = _lib.SSFrame()
    cam = _cam()
    out = ctypes.c_int32()
    # capacity smaller than the pair count
    assert L.ss_sort(ctypes.byref(cam), ctypes.byref(p), 0, 101, ctypes.byref(out),
                     None) == _lib.SS_ERR_WORKSPACE
    p.capacity = 1 << 33
    assert L.ss_sort(ctypes.byref(cam), ctypes.byref(p), 0, 1 << 32, ctypes.byref(out),
                     None) == _lib.SS_ERR_OVERFLOW
    assert L.ss_sort(ctypes.byref(cam), ctypes.byref(p), 2, 5, ctypes.byref(out),
                     None) == _lib.SS_ERR_INVALID_ARG
    assert L.ss_blend(ctypes.byref(cam), ctypes.byref(f), ctypes.byref(p), 0, None,
                      None) == _lib.SS_ERR_INVALID_ARG


def test_ctypes_layouts_match_the_header(tmp_path):
    """Every ctypes struct has the size and field offsets gcc gives the header's."""
    import shutil
    import subprocess

    from paper_2412_00578_amd import _lib
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    structs = {"ss_constants": _lib.SSConstants, "ss_camera": _lib.SSCamera,
               "ss_gaussians": _lib.SSGaussians, "ss_frame": _lib.SSFrame,
               "ss_frame_info": _lib.SSFrameInfo, "ss_frame_counts": _lib.SSFrameCounts,
               "ss_batch_item": _lib.SSBatchItem,
               "ss_batch_info": _lib.SSBatchInfo, "ss_pairs": _lib.SSPairs,
               "ss_grads": _lib.SSGrads, "ss_stage_events": _lib.SSStageEvents}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "speedysplat.h"',
             "int main(void) {"]
    want = []
    for cname, cls in structs.items():
        lines.append(f'printf("%zu\\n", sizeof({cname}));')
        want.append(ctypes.sizeof(cls))
        for fname, _ in cls._fields_:
            lines.append(f'printf("%zu\\n", offsetof({cname}, {fname}));')
            want.append(getattr(cls, fname).offset)
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o",
                    str(exe)], check=True)
    got = [int(x) for x in subprocess.run([str(exe)], check=True, capture_output=True,
                                          text=True).stdout.split()]
    assert got == want
