"""The ctypes structures of the binding against the C headers: a host C program compiled with gcc
prints sizeof and offsetof of every field the binding declares, and each must match the ctypes
layout (a mismatch would make the library read or write past a caller's structure)."""
import ctypes
import os
import shutil
import subprocess

import pytest

from paper_2603_10711_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

STRUCTS = [("scp_problem_desc", B.ProblemDesc), ("admm_params", B.AdmmParams), ("scp_params", B.ScpParams),
           ("scp_tune_entry", B.TuneEntry), ("scp_server_config", B.ServerConfig),
           ("scp_server_stats", B.ServerStats)]


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")
def test_ctypes_layout_matches_headers(tmp_path):
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "scp.h"', '#include "scp_serve.h"',
             "int main(void) {"]
    for cname, cls in STRUCTS:
        lines.append(f'  printf("{cname} . %zu %zu\\n", (size_t)sizeof({cname}), (size_t)0);')
        for fname, _ in cls._fields_:
            lines.append(f'  printf("{cname} {fname} %zu %zu\\n", (size_t)offsetof({cname}, {fname}), '
                         f"(size_t)sizeof((({cname}*)0)->{fname}));")
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-Wall", "-Werror", "-I" + os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {(c, f): (int(a), int(b)) for c, f, a, b in (l.split() for l in out if l)}
    for cname, cls in STRUCTS:
        assert got[(cname, ".")][0] == ctypes.sizeof(cls), cname
        for fname, ftype in cls._fields_:
            off, size = got[(cname, fname)]
            assert (off, size) == (getattr(cls, fname).offset, ctypes.sizeof(ftype)), (cname, fname)
