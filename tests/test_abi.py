"""The C-ABI library loads without a GPU and exports every entry point that
include/bamg.h declares. No compute call is made here."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bamg.h")
LIB = os.path.join(ROOT, "paper_1402_4005_amd", "libbamg.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    names = re.findall(r"^[A-Za-z_][\w \*]*?\b(bamg_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for core in ("bamg_setup", "bamg_vcycle", "bamg_gmres_solve", "bamg_destroy",
                 "bamg_default_options", "bamg_status_string"):
        assert core in names
    assert len(names) >= 15


@pytest.mark.skipif(not os.path.exists(LIB), reason="libbamg.so not built (run build())")
def test_library_exports_every_declared_symbol():
    import torch  # noqa: F401  (loads the HIP runtime the library links against)
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libbamg.so not built (run build())")
def test_host_only_entry_points():
    # default options are the paper's standard parameters (Section 7:
    # r = 8, 3 + 3 weighted-Jacobi sweeps with omega = 0.7, c = 4)
    import paper_1402_4005_amd as bamg
    o = bamg.default_options()
    assert (o.r, o.nu_pre, o.nu_post, o.max_interp, o.setup_cycles) == (8, 3, 3, 4, 1)
    assert o.omega == 0.7
    lib = bamg.lib()
    msgs = {c: lib.bamg_status_string(c) for c in range(-9, 2)}
    assert all(msgs.values()) and len(set(msgs.values())) == len(msgs)
    # a null handle and null arguments are rejected on the host
    assert lib.bamg_default_options(None) == -1
    assert lib.bamg_setup(None, None, None, None, None, None) == -1
