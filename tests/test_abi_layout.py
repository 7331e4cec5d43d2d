"""Host-only check of the C ABI's struct layouts: a C program built with the
system compiler against include/graver.h prints sizeof and offsetof of every
field the ctypes binding declares, and each must equal the binding's.  A
field added to a struct on one side only, a reordering or a padding change
fails here (no GPU needed)."""
import ctypes
import os
import shutil
import subprocess

import pytest

from paper_2412_13576_amd import graver as G

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# C typedef -> ctypes mirror in the binding
STRUCTS = [
    ("graver_problem", G.Problem),
    ("graver_objective", G.ObjectiveC),
    ("graver_extract_params", G.ExtractParams),
    ("graver_state", G.State),
    ("graver_extract_stats", G.ExtractStats),
    ("graver_augment_params", G.AugmentParams),
    ("graver_init_params", G.InitParams),
    ("graver_batch_params", G.BatchParams),
    ("graver_batch_stats", G.BatchStats),
    ("graver_server_params", G.ServerParams),
    ("graver_request", G.RequestC),
    ("graver_result", G.ResultC),
    ("graver_solve_params", G.SolveParams),
    ("graver_solve_stats", G.SolveStats),
]


def _c_layout(tmp_path):
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "graver.h"', "int main(void) {"]
    for cname, cls in STRUCTS:
        lines.append(f'  printf("{cname} sizeof %zu\\n", sizeof({cname}));')
        for fname, _ in cls._fields_:
            lines.append(f'  printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True,
                   capture_output=True, text=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    return {tuple(line.split()[:2]): int(line.split()[2]) for line in out.splitlines()}


def test_ctypes_mirrors_have_the_c_layout(tmp_path):
    c = _c_layout(tmp_path)
    for cname, cls in STRUCTS:
        assert c[(cname, "sizeof")] == ctypes.sizeof(cls), cname
        for fname, _ in cls._fields_:
            assert c[(cname, fname)] == getattr(cls, fname).offset, f"{cname}.{fname}"


def test_extract_params_form_and_stats_fields():
    """The extraction's form selector and the sparse form's statistics are
    the last fields of their structs, after every older field."""
    names = [f for f, _ in G.ExtractParams._fields_]
    assert names[-1] == "form"
    assert G.extract_params(1, 1).form == G.GRAVER_FORM_AUTO
    assert G.extract_params(1, 1, form=G.GRAVER_FORM_SPARSE).form == 2
    st = [f for f, _ in G.ExtractStats._fields_]
    assert st[-2:] == ["row_entries", "row_slots"]
