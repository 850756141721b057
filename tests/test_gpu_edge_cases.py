"""GPU parity on the degenerate and boundary cases of the method.

* isoviscous domains (no inclusion, or an inclusion with the background
  viscosity): no interface vertex, so the interface form is the gradient
  (vector-Laplacian) form on every row (eq. equivalence-stencil, Sec. 2.2);
* two phases with equal viscosity: an interface vertex needs a viscosity
  jump, not a phase change (reading of the remark at the end of Sec. 2.2);
* an inclusion cut by the domain boundary: interface vertices on Dirichlet
  faces, truncated element loops;
* the smallest lattices (9^3 and 9^2: one special vertex ring around a 7^3 /
  7^2 interior), where several XCD row slabs are empty.

Tolerances as in the operator and smoother parity tests: applies
1e-12 x max(|K||x|), one smoothing step 1e-11 relative."""
import numpy as np
import pytest

import iss_inputs
from oracle import assemble, multigrid as mg
from tests.gpu_common import abs_scale, assert_close_scaled, gpu_problem, to_dev, to_host

pytestmark = pytest.mark.gpu


def _w(dim, levels, inclusions, mu, macro=1, coarse=None):
    return dict(name="edge", dim=dim, macro=macro, levels=levels,
                coarse=min(levels, 3) if coarse is None else coarse,
                n=macro * 2 ** levels, inclusions=inclusions, mu=mu, buoyant=[])


def _sphere(c, r, phase=1):
    return {"kind": "sphere", "center": tuple(c), "radius": r, "phase": phase}


CASES = {
    "no-inclusion-3d": _w(3, 4, [], [1.0]),
    "same-mu-3d": _w(3, 4, [_sphere((0.5, 0.5, 0.5), 0.3)], [2.0, 2.0]),
    "same-mu-two-phases-3d": _w(3, 4, [_sphere((0.4, 0.5, 0.5), 0.25), _sphere((0.6, 0.5, 0.5), 0.25, 2)],
                                [1.0, 50.0, 50.0]),
    "boundary-cut-3d": _w(3, 4, [_sphere((0.5, 0.5, 0.0), 0.35), _sphere((1.0, 1.0, 1.0), 0.4)], [1.0, 300.0]),
    "boundary-cut-ragged-3d": _w(3, 3, [_sphere((0.0, 0.3, 0.6), 0.45)], [1.0, 30.0], macro=3),
    "smallest-3d": _w(3, 3, [_sphere((0.5, 0.5, 0.5), 0.3)], [1.0, 100.0]),
    "smallest-2d": _w(2, 3, [{"kind": "halfspace", "axis": 1, "threshold": 0.4, "phase": 1}], [1.0, 10.0]),
    "no-inclusion-2d": _w(2, 5, [], [3.0]),
}


@pytest.fixture(scope="module", params=sorted(CASES))
def case(request):
    w = CASES[request.param]
    P = gpu_problem(w)
    D = assemble.Discretisation(w["dim"], w["n"], w["inclusions"], w["mu"])
    yield request.param, w, P, D
    P.close()


def test_classification(case):
    name, w, P, D = case
    cls, nif, nbd = P.vertex_class()
    assert nif == int(D.interface.sum())
    if name.startswith("no-inclusion") or name == "same-mu-3d":
        assert nif == 0
    if name == "same-mu-two-phases-3d":
        # the two touching spheres share one viscosity: only the outer
        # surface of their union is an interface
        assert nif > 0


@pytest.mark.parametrize("form", ["gradient", "strain", "interface"])
def test_apply_parity(case, form):
    import torch
    name, w, P, D = case
    x = iss_inputs.random_vector(w["dim"], w["n"], seed=41)
    K = D.stokes(form)
    y = torch.empty_like(to_dev(x))
    P.apply(form, to_dev(x), y, block="full")
    assert_close_scaled(to_host(y), K @ x, abs_scale(K, x), 1e-12, "%s/%s" % (name, form))


def test_interface_equals_gradient_without_jumps(case):
    """Without a viscosity jump the two forms are the same operator
    (isoviscous rows use the same bulk stencils, so those agree exactly;
    mixed-phase rows with equal viscosities agree to rounding)."""
    import torch
    name, w, P, D = case
    if D.interface.any():
        pytest.skip("has interface vertices")
    xh = iss_inputs.random_vector(w["dim"], w["n"], seed=42)
    x = to_dev(xh)
    yi, yg = torch.empty_like(x), torch.empty_like(x)
    P.apply("interface", x, yi, block="full")
    P.apply("gradient", x, yg, block="full")
    K = D.stokes("gradient")
    assert_close_scaled(to_host(yi), to_host(yg), abs_scale(K, xh), 1e-14, name)
    if name.startswith("no-inclusion"):
        assert torch.equal(yi, yg)


@pytest.mark.parametrize("form", ["strain", "interface"])
def test_smoother_step_parity(case, form):
    name, w, P, D = case
    lv = mg.Level(w["dim"], w["n"], w["inclusions"], w["mu"], form)
    x = iss_inputs.random_vector(w["dim"], w["n"], seed=43)
    b = iss_inputs.random_rhs(w["dim"], w["n"], seed=44)
    xg = to_dev(x)
    P.smooth(form, xg, to_dev(b), nsteps=1)
    ref = mg.smooth(lv, x, b, 1)
    err = np.abs(to_host(xg) - ref).max() / max(np.abs(ref).max(), 1e-300)
    assert err < 1e-11, (name, form, err)


@pytest.mark.parametrize("form", ["strain", "interface"])
@pytest.mark.parametrize("path", [dict(merge_max_n=0), dict(merge_max_n=0, spec_wide_min=0)],
                         ids=["large", "large-wide"])
def test_smoother_step_parity_large_path(case, form, path):
    """The same step through the kernels of the levels above 65^3 (separate
    bulk and special launches, grouped pressure pass, one-wave or 256-thread
    pressure special groups)."""
    name, w, _, D = case
    P = gpu_problem(w, **path)
    lv = mg.Level(w["dim"], w["n"], w["inclusions"], w["mu"], form)
    x = iss_inputs.random_vector(w["dim"], w["n"], seed=46)
    b = iss_inputs.random_rhs(w["dim"], w["n"], seed=47)
    xg = to_dev(x)
    P.launch_counts(reset=True)
    P.smooth(form, xg, to_dev(b), nsteps=2)
    c = P.launch_counts()
    assert c["gs_vel_merged"] == c["p_rhs_merged"] == c["gs_p_merged"] == 0, c
    assert c["p_rhs_grouped"] == 2, c
    ref = mg.smooth(lv, x, b, 2)
    err = np.abs(to_host(xg) - ref).max() / max(np.abs(ref).max(), 1e-300)
    assert err < 1e-11, (name, form, err)
    P.close()


def test_zero_input_gives_zero(case):
    import torch
    name, w, P, D = case
    x = torch.zeros(P.vector_size(), dtype=torch.float64, device="cuda")
    y = torch.full_like(x, 7.0)
    P.apply("interface", x, y, block="full")
    assert torch.count_nonzero(y).item() == 0


def test_call_errors_and_not_converged():
    """Bad form, precision or level: ISS_E_INVAL and no device work; a solve
    that hits maxit returns ISS_E_NOTCONV with its history filled."""
    import ctypes
    import torch
    from paper_1604_07994_amd import binding
    w = CASES["boundary-cut-3d"]
    P = gpu_problem(w, outer="fgmres")
    L = binding.lib()
    x = torch.zeros(P.vector_size(), dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    xp, yp = ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr())
    assert L.iss_apply(P._h, 7, 1, w["levels"], 0, xp, yp, None) == -1
    assert L.iss_apply(P._h, 2, 1, w["levels"], 9, xp, yp, None) == -1
    assert L.iss_apply(P._h, 2, 1, w["levels"] + 1, 0, xp, yp, None) == -1
    assert L.iss_apply(P._h, 2, 5, w["levels"], 0, xp, yp, None) == -1
    b = to_dev(iss_inputs.random_rhs(3, w["n"], seed=45))
    info = P.solve("interface", x, b, rtol=1e-14, maxit=2, raise_on_fail=False)
    assert info["status"] == -3 and info["iterations"] == 2
    assert len(info["history"]) == 3 and info["history"][-1] < info["history"][0]
    P.close()
