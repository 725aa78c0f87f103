"""C-ABI checks that need no GPU: the library loads, exports every declared symbol, and fails
cleanly on the host-side error paths."""
import ctypes as C
import os
import re

import pytest

from paper_2410_05095_amd import _native as N

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(rc_\w+)\s*\(", text))
    return names


def test_library_exports_every_declared_symbol():
    L = N.lib()
    names = declared_functions()
    assert len(names) >= 15
    for name in names:
        assert hasattr(L, name), name
    # the binding declares a signature for each of them
    assert names == set(N.SIGNATURES)


def test_status_strings():
    L = N.lib()
    for code in range(-8, 1):
        s = L.rc_status_string(code).decode()
        assert s and s != "unknown status"
    assert L.rc_status_string(-99).decode() == "unknown status"
    assert L.rc_version() >= 10000


def test_null_arguments_rejected():
    L = N.lib()
    assert L.rc_create(None, 0, None) == -1
    assert L.rc_destroy(None) == -1
    assert L.rc_set_stream(None, None) == -1
    assert L.rc_get_last_error(None) == -1
    assert L.rc_scene_create(None, None, None) == -1
    assert L.rc_bvh_build(None, None, None) == -1
    assert L.rc_bvh_refit(None, None) == -1
    assert L.rc_render(None, None, None, None, 0, None, None, None) == -1
    assert L.rc_get_stage_times(None, None) == -1
    assert L.rc_camera_rays(None, None, None, None) == -1


def test_no_device_is_a_hip_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    L = N.lib()
    h = C.c_void_p()
    assert L.rc_create(C.byref(h), 0, None) == -4   # RC_ERR_HIP
    assert not h.value


def test_binding_refuses_without_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(RuntimeError):
        N.Context(0)
