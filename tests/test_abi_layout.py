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


def _prototypes():
    """name -> list of parameter type strings, from every prototype in the header."""
    import re
    text = open(os.path.join(ROOT, "include", "iim.h")).read()
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    out = {}
    for m in re.finditer(r"\b(?:int|int64_t|const char\s*\*)\s+(iim_\w+)\s*\(([^)]*)\)\s*;", text):
        params = [p.strip() for p in m.group(2).split(",")]
        if params == ["void"]:
            params = []
        # drop the parameter name: the type is everything before the last identifier
        types = []
        for p in params:
            t = re.sub(r"\b\w+\s*$", "", p).strip() if re.search(r"[\w\*]\s+\w+$", p) else p
            types.append(" ".join(t.replace("*", " * ").split()))
        out[m.group(1)] = types
    return out


_SCALARS = {"int32_t": C.c_int32, "int64_t": C.c_int64, "uint64_t": C.c_uint64, "double": C.c_double,
            "float": C.c_float, "int": C.c_int}
_POINTEES = {"double": C.c_double, "float": C.c_float, "int32_t": C.c_int32, "int64_t": C.c_int64}


def test_argument_types_match_header():
    protos = _prototypes()
    L = iim.lib()
    checked = 0
    for name in iim.EXPORTS:
        fn = getattr(L, name)
        if fn.argtypes is None:
            continue
        types = protos[name]
        assert len(types) == len(fn.argtypes), (name, types, fn.argtypes)
        for ct, at in zip(types, fn.argtypes):
            if "*" in ct:
                # a pointer: the binding passes a pointer of the same pointee
                # size (or an untyped / string / structure pointer)
                assert at in (C.c_void_p, C.c_char_p) or hasattr(at, "_type_") and not isinstance(at._type_, str) \
                    or issubclass(at, C._Pointer), (name, ct, at)
                base = ct.replace("const", "").replace("*", "").split()
                if issubclass(at, C._Pointer) and len(base) == 1 and base[0] in _POINTEES \
                        and ct.count("*") == 1:
                    assert C.sizeof(at._type_) == C.sizeof(_POINTEES[base[0]]), (name, ct, at)
            else:
                base = ct.replace("const", "").split()[-1]
                if base in _SCALARS:
                    assert C.sizeof(at) == C.sizeof(_SCALARS[base]), (name, ct, at)
                    assert (at in (C.c_double, C.c_float)) == (base in ("double", "float")), (name, ct, at)
            checked += 1
    assert checked > 100
