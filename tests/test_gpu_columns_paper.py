"""The viscosity-columns comparison of Sec. 4 (stabilised P1-P1) on the GPU,
against the values the paper prints (tests/golden/columns_p1p1.json).

For levels 2-4 (17^3 to 65^3 vertices) the discrete solutions of the
strain, interface (stencil-modified) and gradient forms are computed with
FGMRES to 1e-11 and compared on the same level in the relative velocity L2
norm (M from the library's force load) and the relative energy norm
||v||_V^2 = a_sym(v, v) (the library's strain apply).  The pressure norm is
not formed (no weighted pressure mass in the library).

The paper leaves the stabilisation constant and the split of its macro
cubes open, so the values are not expected to agree digit for digit; what
the table fixes, and what is checked, is the behaviour: the stencil-modified
solution converges to the strain solution at second order in L2 and first
order in the energy norm, the gradient solution keeps a difference of about
2% in L2 that does not vanish under refinement, and every value lies within
a factor 4 of the printed one."""
import json
import os

import numpy as np
import pytest

import iss_inputs
from tests.gpu_common import small_workload, to_dev

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "columns_p1p1.json")
LEVELS = (2, 3, 4)


def _solutions(level):
    import torch
    from paper_1604_07994_amd import Problem
    w = small_workload("columns_3d", level)
    P = Problem.from_workload(w, outer="fgmres", restart=60, coarse_mu="average", nu1=3, nu2=3, nu_inc=2)
    f = to_dev(np.ascontiguousarray(iss_inputs.column_force(3, w["n"]).ravel()))
    b = torch.empty(P.vector_size(), dtype=torch.float64, device="cuda")
    P.rhs_nodal_force(f, b)
    out = {}
    for form in ("strain", "interface", "gradient"):
        x = torch.zeros_like(b)
        info = P.solve(form, x, b, rtol=1e-11, maxit=300)
        assert info["relres"] <= 1e-11, (form, info)
        out[form] = x
    return P, out


def _norms(P, e):
    """(||e_u||_0, ||e_u||_V) of the velocity part of e."""
    import torch
    N = P.num_vertices()
    m = torch.empty_like(e)
    P.rhs_nodal_force(e[:3 * N].contiguous(), m)
    y = torch.empty_like(e)
    P.apply("strain", e, y, block="velocity")
    l2 = float(torch.dot(e[:3 * N], m[:3 * N]))
    en = float(torch.dot(e[:3 * N], y[:3 * N]))
    return np.sqrt(l2), np.sqrt(en)


@pytest.fixture(scope="module")
def differences():
    res = {}
    for lvl in LEVELS:
        P, x = _solutions(lvl)
        ref = _norms(P, x["strain"])
        for form in ("interface", "gradient"):
            d = _norms(P, x[form] - x["strain"])
            res[(form, lvl)] = {"l2": d[0] / ref[0], "V": d[1] / ref[1]}
        P.close()
    print("columns differences vs strain:", {"%s/%d" % k: v for k, v in res.items()})
    return res


def test_stencil_form_converges_to_strain_form(differences):
    with open(GOLDEN) as fh:
        paper = json.load(fh)["interface_vs_strain"]
    l2 = [differences[("interface", l)]["l2"] for l in LEVELS]
    en = [differences[("interface", l)]["V"] for l in LEVELS]
    r2 = np.log2(np.array(l2[:-1]) / np.array(l2[1:]))
    rv = np.log2(np.array(en[:-1]) / np.array(en[1:]))
    # printed rates: L2 1.79, 1.94; energy 1.02, 1.00
    assert np.all(r2 >= 1.6), (l2, r2)
    assert np.all(rv >= 0.8), (en, rv)
    for l in LEVELS:
        for key in ("l2", "V"):
            ratio = differences[("interface", l)][key] / paper[str(l)][key]
            assert 0.25 <= ratio <= 4.0, (l, key, ratio)


def test_gradient_form_keeps_an_inconsistency(differences):
    with open(GOLDEN) as fh:
        paper = json.load(fh)["gradient_vs_strain"]
    l2 = [differences[("gradient", l)]["l2"] for l in LEVELS]
    # printed: 7.5e-2, 3.0e-2, 2.1e-2, then 2.0e-2 at levels 5 and 6
    assert l2[-1] >= 1e-2, l2
    assert l2[-2] / l2[-1] < 1.5, l2
    for l in LEVELS:
        assert l2[LEVELS.index(l)] > 2 * differences[("interface", l)]["l2"]
        for key in ("l2", "V"):
            ratio = differences[("gradient", l)][key] / paper[str(l)][key]
            assert 0.25 <= ratio <= 4.0, (l, key, ratio)


@pytest.mark.parametrize("form", ["interface", "strain", "gradient"])
def test_columns_rates_in_the_paper_configuration(form):
    """Sec. 5 multigrid on the columns problem (33^3 over 9^3): V(3,3) with
    two more steps per coarser level, omega 0.3, the strain form on the
    coarsest level with the modified momentum right-hand side.  The
    asymptotic rate (200 rescaled cycles) stays in the paper's range
    (0.24-0.30 at levels 5-8) below 0.35; for the interface and gradient
    forms the naive swap (no modification) is slower."""
    import torch
    from paper_1604_07994_amd import Problem
    w = small_workload("columns_3d", 3)
    x0 = to_dev(iss_inputs.random_vector(3, w["n"], seed=157, bc="freeslip"))
    kw = dict(outer="richardson", omega=0.3, nu1=3, nu2=3, nu_inc=2, coarse_mu="average", coarse_form="strain")
    P = Problem.from_workload(w, coarse_rhs_mod=True, **kw)
    rate = P.asymptotic_rate(form, x0.clone(), iters=200)[-1]
    P.close()
    assert rate < 0.35, (form, rate)
    if form != "strain":
        Pn = Problem.from_workload(w, **kw)
        naive = Pn.asymptotic_rate(form, x0.clone(), iters=200)[-1]
        Pn.close()
        assert naive > rate + 0.02, (form, rate, naive)
