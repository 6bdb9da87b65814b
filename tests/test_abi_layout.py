"""The C ABI's structures as the header lays them out (compiled with the
host C compiler) against the binding's ctypes structures: the size of every
structure and the offset of every field.  A drift between the two would let
the library read or write past the caller's buffers."""
import ctypes as C
import os
import shutil
import subprocess

import pytest

import paper_2109_13628_amd as iim

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
STRUCTS = {"iim_grid_desc": iim.GridDesc, "iim_body_desc": iim.BodyDesc, "iim_solver_opts": iim.SolverOpts,
           "iim_step_stats": iim.StepStats, "iim_info": iim.Info, "iim_geometry_view": iim.GeometryView,
           "iim_counters": iim.Counters, "iim_net_desc": iim.NetDesc, "iim_batch_tuning": iim.BatchTuning,
           "iim_batch_stats": iim.BatchStats}


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no host C compiler")
def test_struct_layouts_match_header(tmp_path):
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "iim.h"', "int main(void) {"]
    for cname, py in STRUCTS.items():
        lines.append('  printf("%s %%zu\\n", sizeof(%s));' % (cname, cname))
        for f in py._fields_:
            lines.append('  printf("%s.%s %%zu\\n", offsetof(%s, %s));' % (cname, f[0], cname, f[0]))
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    checked = 0
    for line in filter(None, out):
        name, value = line.split()
        if "." in name:
            cname, field = name.split(".")
            got = getattr(STRUCTS[cname], field).offset
        else:
            got = C.sizeof(STRUCTS[name])
        assert got == int(value), (name, int(value), got)
        checked += 1
    assert checked == len(STRUCTS) + sum(len(p._fields_) for p in STRUCTS.values())
