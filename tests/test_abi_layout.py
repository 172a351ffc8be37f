"""The ctypes mirrors of the C structs in include/tmotif.h have the C layout:
a small C program built with the host compiler prints the size of every
struct and the offset of every field, which must equal ctypes' figures."""
from __future__ import annotations

import ctypes
import os
import shutil
import subprocess

import pytest

from paper_2310_02800_amd import _native as N

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PAIRS = [(N.EdgePred, "tm_edge_pred"), (N.MotifDesc, "tm_motif_desc"), (N.RootRange, "tm_root_range"),
         (N.ServerCfg, "tm_server_cfg"), (N.Query, "tm_query"), (N.Result, "tm_result"),
         (N.GraphInfo, "tm_graph_info")]


def c_layout(tmp_path):
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "tmotif.h"', "int main(void) {"]
    for cls, cname in PAIRS:
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for f in cls._fields_:
            lines.append(f'  printf("{cname} {f[0]} %zu\\n", offsetof({cname}, {f[0]}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"), "-I", "/opt/rocm/include",
                    str(src), "-o", str(exe)], check=True, capture_output=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    return {tuple(l.split()[:2]): int(l.split()[2]) for l in out.splitlines()}


@pytest.mark.skipif(shutil.which("gcc") is None or not os.path.isdir("/opt/rocm/include"),
                    reason="needs gcc and the HIP headers")
def test_ctypes_mirrors_match_c_layout(tmp_path):
    c = c_layout(tmp_path)
    for cls, cname in PAIRS:
        assert c[(cname, "size")] == ctypes.sizeof(cls), cname
        for f in cls._fields_:
            assert c[(cname, f[0])] == getattr(cls, f[0]).offset, (cname, f[0])
