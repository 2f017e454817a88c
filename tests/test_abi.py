"""The C-ABI library loads and exports every symbol the headers declare (CPU:
no compute calls)."""
import ctypes
import glob
import os
import re

import pytest

from paper_2001_07428_amd import jlanczos

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        txt = open(h).read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        names |= set(re.findall(r"^\s*(?:const\s+char\s*\*|jl_status)\s+(jl_\w+)\s*\(", txt, flags=re.M))
    return names


def test_headers_declare_the_binding_exports():
    declared = _declared()
    assert declared, "no declarations parsed"
    assert declared == set(jlanczos.EXPORTS)


def test_library_exports_every_declared_symbol():
    if not os.path.exists(jlanczos.LIB_PATH):
        pytest.fail("libjlanczos.so is not built (python -m paper_2001_07428_amd.build)")
    lib = ctypes.CDLL(jlanczos.LIB_PATH)
    for name in _declared():
        assert hasattr(lib, name), name


def test_status_strings_without_gpu():
    lib = jlanczos.load_library()
    assert lib.jl_status_string(0) == b"ok"
    assert lib.jl_status_string(-3) == b"workspace too small"
    # workspace queries that need no device
    nb = ctypes.c_size_t()
    assert lib.jl_ritz_workspace_bytes(10, ctypes.byref(nb)) == 0 and nb.value > 0
    assert lib.jl_reorth_pass_workspace_bytes(7, 3, ctypes.byref(nb)) == jlanczos.JL_EINVAL  # odd n
    assert lib.jl_reorth_pass_workspace_bytes(2000, 12, ctypes.byref(nb)) == 0
