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
    return sorted(set(re.findall(r"\b(iss_[a-z0-9_]+)\s*\(", src)))


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
    assert opt.coarse_form == -1 and opt.mid_form == -1
    assert opt.merge_max_n == 64 and opt.spec_wide_min == 65536 and opt.cycles == 1
    assert opt.bc == 0 and opt.split_align == 0 and opt.coarse_solver == 0
    assert opt.minres_iters == 30 and opt.minres_cg == 5


def _create(L, binding, dim=3, macro=1, levels=2, coarse=1, incs=(), mu=(1.0,), opt=None):
    h = ctypes.c_void_p()
    arr = binding.inclusions_to_c(list(incs))
    m = (ctypes.c_double * max(1, len(mu)))(*mu)
    rc = L.iss_problem_create(dim, macro, levels, coarse, arr, len(incs), m, len(mu),
                              None if opt is None else ctypes.byref(opt), ctypes.byref(h))
    return rc, L.iss_last_error().decode()


@pytest.mark.parametrize("kw,msg", [
    (dict(macro=0), "macro"),
    (dict(levels=1, coarse=2), "coarse_level"),
    (dict(coarse=0), "coarse_level"),
    (dict(mu=()), "nphase"),
    (dict(mu=tuple([1.0] * 255)), "nphase"),
    (dict(mu=(1.0, float("inf"))), "viscosities"),
    (dict(mu=(1.0, 0.0)), "viscosities"),
    (dict(incs=[{"kind": "sphere", "center": (0.5, 0.5, 0.5), "radius": 0.2, "phase": 2}], mu=(1.0, 2.0)),
     "phase"),
    (dict(incs=[{"kind": "halfspace", "axis": 3, "threshold": 0.5, "phase": 1}], mu=(1.0, 2.0)), "axis"),
])
def test_problem_create_rejects_bad_arguments(kw, msg):
    """Every argument check of iss_problem_create runs before any device
    call: ISS_E_INVAL (-1) and a message naming the argument."""
    from paper_1604_07994_amd import binding
    L = binding.lib()
    rc, err = _create(L, binding, **kw)
    assert rc == -1 and msg in err, (rc, err)


def test_problem_create_rejects_split_field_beyond_4gib():
    """A 2D lattice that passes the int32 index bound but whose colour-split
    smoother field would exceed 4 GiB (32-bit byte offsets) is rejected
    before any device call: macro 3, 13 refinements (24577^2 vertices)."""
    from paper_1604_07994_amd import binding
    L = binding.lib()
    rc, err = _create(L, binding, dim=2, macro=3, levels=13, coarse=3)
    assert rc == -1 and "4 GiB" in err, (rc, err)


@pytest.mark.parametrize("field,value", [("nu1", -1), ("nu_inc", -2), ("restart", 0), ("outer", 5),
                                         ("coarse_mu", 7), ("coarse_form", 3), ("stab_beta", 0.0),
                                         ("mid_form", -2), ("mid_form", 3), ("merge_max_n", -1),
                                         ("spec_wide_min", -1), ("cycles", 0), ("cycles", 17), ("f16_rms", 0.0),
                                         ("f16_rms", 1e5), ("bc", 2), ("split_align", -1), ("split_align", 65),
                                         ("coarse_solver", 2), ("minres_iters", 0), ("minres_iters", 1001),
                                         ("minres_cg", -1), ("minres_cg", 101)])
def test_problem_create_rejects_bad_options(field, value):
    from paper_1604_07994_amd import binding
    L = binding.lib()
    opt = binding.Options()
    assert L.iss_default_options(ctypes.byref(opt)) == 0
    setattr(opt, field, value)
    rc, err = _create(L, binding, opt=opt)
    assert rc == -1 and "options" in err, (rc, err)


def test_null_arguments_are_rejected():
    from paper_1604_07994_amd import binding
    L = binding.lib()
    assert L.iss_default_options(None) == -1
    mu = (ctypes.c_double * 1)(1.0)
    assert L.iss_problem_create(3, 1, 2, 1, None, 0, mu, 1, None, None) == -1
    assert L.iss_apply(None, 2, 1, 2, 0, None, None, None) == -1
    assert L.iss_solve(None, 2, 0, 1e-8, 10, None, None, None, None) == -1
    assert L.iss_rhs_nodal_force(None, 2, None, None, None) == -1
    assert L.iss_num_elements(None, None) == -1
    assert L.iss_p1p0_apply(None, 2, 1.0, None, None, None) == -1
    assert L.iss_p1p0_flux(None, 1.0, None, None, None) == -1
