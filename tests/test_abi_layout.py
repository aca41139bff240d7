"""The ctypes mirrors of the public structs (paper_1408_6299_amd/_lib.py) have the layout the C
compiler gives include/nkreg.h: every field at the same offset, every struct the same size.
Built with gcc from the header alone; no GPU and no library needed."""
import ctypes
import json
import os
import shutil
import subprocess

import pytest

from paper_1408_6299_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

MIRRORS = {"nkreg_config": _lib.Config, "nkreg_solve_opts": _lib.SolveOpts, "nkreg_solve_report": _lib.SolveReport,
           "nkreg_picard_opts": _lib.PicardOpts, "nkreg_beta_search_opts": _lib.BetaSearchOpts,
           "nkreg_beta_search_report": _lib.BetaSearchReport}


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_ctypes_structs_match_the_c_header(tmp_path):
    lines = ['#include "nkreg.h"', "#include <stdio.h>", "#include <stddef.h>", "int main(void) {", '  printf("{");']
    first = True
    for cname, py in MIRRORS.items():
        items = [f'\\"size\\": %zu'] + [f'\\"{f}\\": %zu' for f, _ in py._fields_]
        args = [f"sizeof({cname})"] + [f"offsetof({cname}, {f})" for f, _ in py._fields_]
        sep = "" if first else ", "
        first = False
        lines.append(f'  printf("{sep}\\"{cname}\\": {{{", ".join(items)}}}", {", ".join(args)});')
    lines += ['  printf("}\\n");', "  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True,
                   capture_output=True, timeout=120)
    got = json.loads(subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout)
    for cname, py in MIRRORS.items():
        assert got[cname]["size"] == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[cname][f] == getattr(py, f).offset, (cname, f)


def test_history_columns_match_the_header():
    text = open(os.path.join(ROOT, "include", "nkreg.h")).read()
    assert f"#define NKREG_HISTORY_COLS {_lib.HISTORY_COLS}" in text
