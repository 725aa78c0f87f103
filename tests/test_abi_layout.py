"""The ctypes structures of the binding have the C header's layout: every struct of include/raycast.h that
the binding mirrors is compiled with gcc, and its size and field offsets are compared with ctypes'
(CPU only; no library call)."""
import ctypes as C
import os
import subprocess
import tempfile

import pytest

from paper_2410_05095_amd import _native as N

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

PAIRS = [("rc_scene_desc", N.RcSceneDesc), ("rc_build_opts", N.RcBuildOpts), ("rc_bvh_stats", N.RcBvhStats),
         ("rc_camera", N.RcCamera), ("rc_point_light", N.RcPointLight), ("rc_rect_light", N.RcRectLight),
         ("rc_render_opts", N.RcRenderOpts), ("rc_outputs", N.RcOutputs), ("rc_view", N.RcView),
         ("rc_tune", N.RcTune), ("rc_stage_times", N.RcStageTimes)]


def c_layout():
    """{struct: (size, {field: offset})} from a C program compiled against the header."""
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "raycast.h"', "int main(void) {"]
    for cname, cls in PAIRS:
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in cls._fields_:
            lines.append(f'printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["return 0;", "}"]
    with tempfile.TemporaryDirectory() as d:
        src, exe = os.path.join(d, "layout.c"), os.path.join(d, "layout")
        with open(src, "w") as f:
            f.write("\n".join(lines))
        subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), src, "-o", exe], check=True)
        out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout
    res = {}
    for line in out.splitlines():
        s, f, v = line.split()
        entry = res.setdefault(s, [0, {}])
        if f == "size":
            entry[0] = int(v)
        else:
            entry[1][f] = int(v)
    return res


@pytest.mark.skipif(subprocess.run(["which", "gcc"], capture_output=True).returncode != 0, reason="no gcc")
def test_ctypes_structs_match_header():
    lay = c_layout()
    for cname, cls in PAIRS:
        size, offs = lay[cname]
        assert C.sizeof(cls) == size, (cname, C.sizeof(cls), size)
        for fname, _ in cls._fields_:
            assert getattr(cls, fname).offset == offs[fname], (cname, fname)
