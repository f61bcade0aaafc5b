"""The C-ABI library loads and exports every function the public header declares (no GPU)."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tt_fv.h")
LIB = os.path.join(ROOT, "paper_2408_03483_amd", "libttfv.so")


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = re.findall(r"\b(tt_[a-z_0-9]+)\s*\(", txt)
    return sorted(set(names))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for required in ("tt_fv_init", "tt_fv_step", "tt_round", "tt_cross", "tt_reciprocal"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libttfv.so not built")
def test_library_exports_every_declared_symbol():
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r"\bT (tt_[a-z_0-9]+)", out))
    missing = [n for n in declared_functions() if n not in exported]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libttfv.so not built")
def test_binding_loads_without_gpu():
    from paper_2408_03483_amd import ttfv
    L = ttfv.load_library()
    for n in declared_functions():
        assert hasattr(L, n)
    assert set(ttfv.EXPORTS) <= set(declared_functions())
