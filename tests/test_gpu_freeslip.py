"""GPU parity of the free-slip boundary condition (eq. boundary) on the
viscosity-columns problem of Sec. 4 (mu 1 and 10, two resolved columns,
free-slip on the whole boundary), through the C ABI.

Free-slip fixes the normal velocity component on each face; the tangential
components of boundary vertices are unknowns whose rows the special
(element-loop) kernels form with the full element rows of the form.  The
oracle is assembled with the same fixed set (mesh.fixed_velocity).

Tolerances as for the no-slip tests: applies and residuals 1e-12 of
max(|K| |x|), smoothing steps 1e-11 and V-cycles 1e-10 of max |x|, the force
load 1e-14 of max |b| (a sum of at most 24 x 5 products).  Both kernel
shapes run (merged launches; large-level launches with merge_max_n = 0,
also with every colour run padded to 16 entries, split_align = 16)."""
import numpy as np
import pytest

import iss_inputs
from oracle import assemble, multigrid as mg, problem
from tests.gpu_common import abs_scale, assert_close_scaled, gpu_problem, small_workload, to_dev, to_host

pytestmark = pytest.mark.gpu

CASES = [("columns_3d", 2, 2), ("columns_3d", 2, 4), ("square_split_2d", 5, None)]
PATHS = {"merged": {}, "large": dict(merge_max_n=0), "large-aligned": dict(merge_max_n=0, split_align=16)}


def _workload(name, levels, macro):
    w = small_workload(name, levels, macro)
    w["coarse"] = min(w["coarse"], levels - 1)
    w["bc"] = "freeslip"
    return w


@pytest.fixture(scope="module", params=[(c, p) for c in CASES for p in sorted(PATHS)],
                ids=["%s-L%d-m%s-%s" % (c + (p,)) for c in CASES for p in sorted(PATHS)])
def case(request):
    (name, levels, macro), path = request.param
    w = _workload(name, levels, macro)
    P = gpu_problem(w, **PATHS[path])
    assert P.bc == "freeslip"
    yield w, P
    P.close()


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


@pytest.mark.parametrize("block", ["velocity", "full"])
@pytest.mark.parametrize("form", ["gradient", "strain", "interface"])
def test_apply_and_residual_freeslip(case, form, block):
    import torch
    w, P = case
    d, n = w["dim"], w["n"]
    D = assemble.Discretisation(d, n, w["inclusions"], w["mu"], bc="freeslip")
    K = D.stokes(form)
    N = D.N
    if block == "velocity":
        K = K[:d * N][:, :d * N]
    x = iss_inputs.random_vector(d, n, seed=150, bc="freeslip")
    b = iss_inputs.random_rhs(d, n, seed=151, bc="freeslip")
    xg = to_dev(x)
    y = torch.empty_like(xg)
    P.apply(form, xg, y, block=block)
    nv = K.shape[0]
    scale = abs_scale(K, x[:nv])
    assert_close_scaled(to_host(y)[:nv], K @ x[:nv], scale, 1e-12, "%s/%s apply" % (form, block))
    # outputs hold zero on the fixed entries
    yh = to_host(y)
    assert np.all(yh[:d * N][D.fixed.ravel()] == 0)
    if block == "full":
        r = torch.empty_like(y)
        P.residual(form, xg, to_dev(b), r)
        assert_close_scaled(to_host(r), b - K @ x, scale + np.abs(b), 1e-12, "%s residual" % form)


@pytest.mark.parametrize("form", ["gradient", "strain", "interface"])
def test_smoother_steps_freeslip(case, form):
    w, P = case
    d, n = w["dim"], w["n"]
    lv = mg.Level(d, n, w["inclusions"], w["mu"], form, bc="freeslip")
    x = iss_inputs.random_vector(d, n, seed=152, bc="freeslip")
    b = iss_inputs.random_rhs(d, n, seed=153, bc="freeslip")
    xg = to_dev(x)
    P.smooth(form, xg, to_dev(b), nsteps=2)
    xh = to_host(xg)
    assert _rel(xh, mg.smooth(lv, x, b, 2)) < 1e-11, form
    assert np.all(xh[:d * lv.N][lv.disc.fixed.ravel()] == 0)


@pytest.mark.parametrize("coarse_form", [None, "strain"])
@pytest.mark.parametrize("form", ["gradient", "strain", "interface"])
def test_vcycle_freeslip(form, coarse_form):
    """V(3,3) with averaged coarse viscosity; restriction zeroes only the
    fixed components, the coarse solve's free set follows free-slip."""
    for path in sorted(PATHS):
        w = _workload("columns_3d", 2, 4)
        P = gpu_problem(w, coarse_mu="average", coarse_form=coarse_form, **PATHS[path])
        H = mg.Hierarchy(3, w["macro"], w["levels"], w["coarse"], w["inclusions"], w["mu"], form,
                         coarse_mu="average", coarse_form=coarse_form, bc="freeslip")
        x = iss_inputs.random_vector(3, w["n"], seed=154, bc="freeslip")
        b = iss_inputs.random_rhs(3, w["n"], seed=155, bc="freeslip")
        xg = to_dev(x)
        P.vcycle(form, xg, to_dev(b))
        assert _rel(to_host(xg), H.vcycle(w["levels"], x, b)) < 1e-10, (form, path)
        P.close()


@pytest.mark.parametrize("bc", ["noslip", "freeslip"])
@pytest.mark.parametrize("name,levels,macro", [("columns_3d", 2, 2), ("square_split_2d", 4, None)])
def test_nodal_force_load(name, levels, macro, bc):
    import torch
    w = _workload(name, levels, macro)
    w["bc"] = bc
    P = gpu_problem(w)
    d, n = w["dim"], w["n"]
    D = assemble.Discretisation(d, n, w["inclusions"], w["mu"], bc=bc)
    f = iss_inputs.column_force(d, n)
    f[0] += iss_inputs.random_vector(d, n, seed=156, zero_dirichlet=False)[:D.N]
    ref = problem.rhs_from_nodal_force(d, n, D.elems, f.T) * D.free_mask()
    b = torch.full((P.vector_size(),), 7.0, dtype=torch.float64, device="cuda")
    P.rhs_nodal_force(to_dev(np.ascontiguousarray(f.ravel())), b)
    assert np.abs(to_host(b) - ref).max() <= 1e-14 * np.abs(ref).max()
    P.close()


@pytest.mark.parametrize("form", ["strain", "interface", "gradient"])
def test_columns_solve_matches_direct(form):
    """FGMRES with the V-cycle preconditioner on the columns problem at
    9^3 (the oracle's sparse direct solve finishes in a second): the GPU
    solution to 1e-12 agrees with x* = K^-1 b to 1e-9 of max |x*|."""
    import torch
    w = _workload("columns_3d", 2, 2)
    P = gpu_problem(w, outer="fgmres", coarse_mu="average")
    d, n = 3, w["n"]
    D = assemble.Discretisation(d, n, w["inclusions"], w["mu"], bc="freeslip")
    f = iss_inputs.column_force(d, n)
    b = problem.rhs_from_nodal_force(d, n, D.elems, f.T) * D.free_mask()
    lv = mg.Level(d, n, w["inclusions"], w["mu"], form, bc="freeslip")
    xs = mg.direct_solve(lv, b)
    bg = torch.empty(P.vector_size(), dtype=torch.float64, device="cuda")
    P.rhs_nodal_force(to_dev(np.ascontiguousarray(f.ravel())), bg)
    x = torch.zeros_like(bg)
    info = P.solve(form, x, bg, rtol=1e-12, maxit=200)
    assert info["relres"] <= 1e-12
    xh = to_host(x)
    N = D.N
    # the pressure is fixed up to a constant: compare after the oracle's
    # weighted-mean normalisation
    xh = problem.normalise_pressure(xh, d, n, lv.weights)
    assert _rel(xh, xs) < 1e-9, form
    P.close()


@pytest.mark.parametrize("form", ["strain", "interface"])
def test_smoother_step_fp32_freeslip(form):
    """FP32 vectors and arithmetic on the free-slip columns problem, large
    and merged kernels: one step within 1e-5 of max |x| of the FP64 oracle
    run on the same FP32-rounded input (the tolerance of the no-slip FP32
    tests)."""
    import torch
    for path in sorted(PATHS):
        w = _workload("columns_3d", 2, 2)
        P = gpu_problem(w, **PATHS[path])
        lv = mg.Level(3, w["n"], w["inclusions"], w["mu"], form, bc="freeslip")
        x = iss_inputs.random_vector(3, w["n"], seed=158, bc="freeslip").astype(np.float32).astype(np.float64)
        b = iss_inputs.random_rhs(3, w["n"], seed=159, bc="freeslip").astype(np.float32).astype(np.float64)
        xg = to_dev(x, torch.float32)
        P.smooth(form, xg, to_dev(b, torch.float32), nsteps=1)
        assert _rel(to_host(xg), mg.smooth(lv, x, b, 1)) < 1e-5, (form, path)
        P.close()
