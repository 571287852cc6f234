"""The C-ABI library loads and exports every entry point that include/*.h declare.

No compute call is made here (no GPU is needed); argument checks that fail
before any device work are exercised as well.
"""
import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = sorted(glob.glob(os.path.join(ROOT, "include", "*.h")))


def declared_functions():
    names = set()
    for h in HEADERS:
        src = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names |= set(re.findall(r"\b(ls2?_[a-z0-9_]+)\s*\(", src))
    return sorted(names)


def test_header_declares_the_entry_points():
    names = declared_functions()
    for required in ["ls_plan_create", "ls_apply", "ls_plan_destroy", "ls_status_string",
                     "ls2_plan_create", "ls2_apply", "ls2_plan_destroy"]:
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_1804_02297_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("library not built")
    lib = ctypes.CDLL(binding.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    # the binding wraps exactly the declared functions
    assert sorted(s[0] for s in binding.SIGNATURES) == declared_functions()


def test_host_side_argument_checks():
    from paper_1804_02297_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("library not built")
    lib = binding.load()
    assert lib.ls_status_string(0) == b"ok"
    assert lib.ls_status_string(-6) == b"call out of order"
    h = ctypes.c_void_p()
    # NULL descriptor and n < 3 are rejected before any device work
    assert lib.ls_plan_create(None, None, None, ctypes.byref(h)) == -1
    d = binding.PlanDesc(2, 1.0, 1, 0, None)
    assert lib.ls_plan_create(ctypes.byref(d), ctypes.c_void_p(1), None, ctypes.byref(h)) == -1
    assert lib.ls_apply(None, None, None, 1, 0, None) == -1
    assert lib.ls_plan_fft_size(None) == 0
