"""The shared library loads without a GPU and exports every function that
include/*.h declares."""
import ctypes
import glob
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?\w+\s*\**\s*(tn_\w+)\s*\(", text, flags=re.M):
            names.add(m.group(1))
    return names


def test_every_declared_symbol_is_exported():
    import paper_1908_08553_amd as tn
    names = declared()
    assert {"tn_plan_grid", "tn_contract_grid", "tn_last_error"} <= names
    for n in sorted(names):
        assert hasattr(tn.lib, n), n
        assert ctypes.cast(getattr(tn.lib, n), ctypes.c_void_p).value


def test_built_for_gfx950_only():
    import paper_1908_08553_amd as tn
    data = open(tn.library_path, "rb").read()
    assert b"gfx950" in data
