"""The C ABI on the CPU: the in-tree libflod.so loads and exports every function declared in
include/flod.h; host-only helpers and argument validation work without a device call."""
import ctypes as C
import json
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "flod.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = set()
    for m in re.finditer(r"^\s*(?!typedef)[A-Za-z_][\w\s\*]*?\b(flod_\w+)\s*\(", text, flags=re.M):
        names.add(m.group(1))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    from paper_2408_12894_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2408_12894_amd import build
        build.build()
    return _lib.load()


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("flod_render_level", "flod_render_selective", "flod_render_backward", "flod_ctx_create"):
        assert must in names
    assert len(names) >= 15


def test_every_declared_symbol_is_exported(lib):
    from paper_2408_12894_amd import _lib
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True, text=True).stdout
    exported = {l.split()[-1] for l in out.splitlines() if " T " in l}
    for name in declared_functions():
        assert name in exported, name
        assert hasattr(lib, name)
    assert set(_lib.EXPORTS) == set(declared_functions())


def test_eq3_and_eq7_host_helpers(lib):
    g = json.load(open(os.path.join(ROOT, "tests", "golden", "flod_paper_constants.json")))
    got = [lib.flod_smin(l, g["L_max"], g["lambda"], g["rho"]) for l in range(1, g["L_max"] + 1)]
    np.testing.assert_allclose(got, g["s_min_per_level"], rtol=1e-7)
    d = lib.flod_dproj(0.2, 1662.769, 1.0)
    assert abs(0.2 * 1662.769 / d - 1.0) < 1e-6


def test_status_strings(lib):
    from paper_2408_12894_amd import _lib
    for code in (0, -1, -2, -3, -4, -5):
        assert len(_lib.status_str(code)) >= 2
    assert _lib.status_str(-99) == "unknown status"
    names = [lib.flod_stage_name(k).decode() for k in range(_lib.NUM_STAGES)]
    assert names == list(_lib.STAGES)


def test_validation_before_any_device_call(lib):
    from paper_2408_12894_amd import _lib
    bad = _lib.FLOD_ERR_INVALID_ARG
    lv = _lib.Level()
    cam = _lib.Camera()
    fr = _lib.Frame()
    bg = (C.c_float * 3)(0, 0, 0)
    assert lib.flod_render_level(None, C.byref(lv), 3, C.byref(cam), bg, C.byref(fr), None) == bad
    assert lib.flod_render_backward(None, None, None, None) == bad
    n64 = C.c_int64(0)
    assert lib.flod_render_merged(None, C.byref(lv), 1, 3, C.byref(cam), bg, C.byref(fr), None) == bad
    assert lib.flod_select_compact(None, C.byref(lv), 1, 1, 1, None, None, None, C.byref(n64), None) == bad
    assert lib.flod_overlap_prune(None, C.byref(lv), 0.1, None, None, C.byref(n64), None) == bad
    assert lib.flod_compact_level(None, C.byref(lv), None, None, C.byref(n64), None) == bad
    assert lib.flod_level_transition(None, C.byref(lv), 0.0, C.byref(lv), None) == bad
    st, gr, hp = _lib.LevelState(), _lib.Grads(), _lib.AdamParams()
    assert lib.flod_adam_step(None, C.byref(st), C.byref(gr), C.byref(st), C.byref(st), 4, C.byref(hp), None) == bad
    assert lib.flod_l1_ssim_forward(None, None, None, 3, 4, 4, 0.2, None, None, None) == bad
    assert lib.flod_l1_ssim_backward(None, None, None, 3, 4, 4, 0.2, None, None, None, None) == bad
    assert lib.flod_l1_loss_forward(None, None, None, 16, None, None) == bad
    assert lib.flod_l1_loss_backward(None, None, None, 16, None, None, None) == bad
    assert lib.flod_ctx_stats(None, None) == bad
    assert lib.flod_ctx_view(None, None) == bad
    assert lib.flod_ctx_set_timing(None, 1) == bad
    assert lib.flod_ctx_trim(None, None) == bad
    # a context pointer is required, and alloc/release must come together
    assert lib.flod_ctx_create(None, 0, _lib.ALLOC_FN(0), _lib.FREE_FN(0), None) == bad
    h = C.c_void_p()
    only_alloc = _lib.ALLOC_FN(lambda u, n, s: None)
    assert lib.flod_ctx_create(C.byref(h), 0, only_alloc, _lib.FREE_FN(0), None) == bad
    assert lib.flod_copy_to_host(None, None, 0) == _lib.FLOD_OK
    assert lib.flod_ctx_workspace_bytes(None) == 0


def test_product_and_oracle_are_independent():
    pkg = os.path.join(ROOT, "paper_2408_12894_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                src = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"^\s*(import|from)\s+oracle\b", src, re.M), f
                assert "liboracle" not in src, f
    osrc = open(os.path.join(ROOT, "oracle", "__init__.py")).read() + open(os.path.join(ROOT, "oracle", "oracle.cpp")).read()
    assert "paper_2408_12894_amd" not in osrc
    assert "libflod" not in osrc
