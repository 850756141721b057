"""The C-ABI library loads and exports every function include/iss.h declares
(no GPU needed: no compute call is made)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "iss.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(iss_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("iss_apply", "iss_residual", "iss_smooth", "iss_vcycle", "iss_solve",
                     "iss_restrict", "iss_prolong_add", "iss_coarse_solve"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_1604_07994_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        pytest.fail("libiss.so is not built (run __graft_entry__.build())")
    L = ctypes.CDLL(binding.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing
    assert sorted(binding.EXPORTS) == declared_functions()


def test_argument_validation_without_gpu():
    """Invalid arguments are rejected before any device work."""
    from paper_1604_07994_amd import binding
    L = binding.lib()
    h = ctypes.c_void_p()
    mu = (ctypes.c_double * 1)(1.0)
    assert L.iss_problem_create(4, 1, 2, 1, None, 0, mu, 1, None, ctypes.byref(h)) == -1
    assert b"dim" in L.iss_last_error()
    assert L.iss_problem_create(3, 1, 2, 3, None, 0, mu, 1, None, ctypes.byref(h)) == -1
    bad = (ctypes.c_double * 1)(-1.0)
    assert L.iss_problem_create(3, 1, 2, 1, None, 0, bad, 1, None, ctypes.byref(h)) == -1
    opt = binding.Options()
    assert L.iss_default_options(ctypes.byref(opt)) == 0
    assert opt.nu1 == 3 and opt.nu2 == 3 and abs(opt.omega - 0.3) < 1e-15
