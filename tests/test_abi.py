"""The C-ABI library loads (without a GPU) and exports every function that
include/*.h declares; the binding's status codes match the header."""
import glob
import os
import re
import subprocess

import pytest

from paper_2005_05398_amd import fm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
lib_built = pytest.mark.skipif(not os.path.exists(fm.LIB_PATH), reason="libfm.so not built")


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?\w+\s*\*?\s*(fm_\w+)\s*\(", text, flags=re.M):
            names.add(m.group(1))
    return names


def test_header_declares_entry_points():
    names = declared_functions()
    for n in ("fm_create_problem", "fm_destroy_problem", "fm_problem_info", "fm_apply_operator",
              "fm_apply_precond", "fm_solve", "fm_last_error"):
        assert n in names


@lib_built
def test_library_exports_every_declared_symbol():
    out = subprocess.run(["nm", "-D", "--defined-only", fm.LIB_PATH], stdout=subprocess.PIPE, text=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if line.strip()}
    missing = declared_functions() - exported
    assert not missing, missing
    L = fm.lib()                      # loads without touching a device
    for n in declared_functions():
        assert hasattr(L, n)


def test_status_codes_match_header():
    text = open(os.path.join(ROOT, "include", "fm.h")).read()
    for name, val in re.findall(r"(FM_E?_?\w+)\s*=\s*(-?\d+)", text):
        if name in fm.STATUS_NAMES.values():
            assert fm.STATUS_NAMES[int(val)] == name
