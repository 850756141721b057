"""GPU parity of the smoother kernels that serve the levels above 65^3.

On levels with n > 64 (129^3 and 257^3 in the benchmark) the Uzawa step of
eq. Uzawa_smooth runs in separate bulk and special launches per colour
phase: the right-hand-side passes (LDS-tiled in 3D: k_vel_rhs_z and
k_p_rhs_z, which also finishes colour 0; k_vel_rhs_s and k_p_rhs_g in 2D),
k_gs_vel_s, k_gs_vel_special_s, k_gs_p_s and k_gs_p_special_s in one-wave or
256-thread workgroups; the bulk rows of applies and residuals take the
LDS-tiled k_apply_z in 3D.  Smaller levels use merged launches.  The option merge_max_n = 0 selects the large-level
kernels on every level, spec_wide_min = 0 sends every pressure special
list to the 256-thread kernel and split_align = 16 pads every colour run of
the split layout to a multiple of 16 entries (the automatic padding of the
large levels, here at small sizes), so these kernels are compared with the
oracle here at sizes the oracle handles (17^3 to 33^3, 33^2, a ragged
25^3), and the host launch counters show which kernels ran.

Tolerances: FP64 as for the merged path (one smoothing step 1e-11, one
V-cycle 1e-10, relative to max |x|).  FP32 (vectors and arithmetic in
FP32): each updated entry is a short sum of products rounded at u = 2^-24
~ 6e-8, and a Gauss-Seidel step carries earlier updates forward; one step
is held to 1e-5 (~170 u) of max |x| against the FP64 oracle run on the
same FP32-rounded input, one V-cycle to 1e-4."""
import itertools

import numpy as np
import pytest

import iss_inputs
from oracle import multigrid as mg
from tests.gpu_common import gpu_problem, small_workload, to_dev, to_host

pytestmark = pytest.mark.gpu

CASES = [("square_split_2d", 5, None), ("sphere_3d", 4, None), ("sinker_3d", 4, None),
         ("sphere_3d", 3, 3)]
PATHS = {"large": dict(merge_max_n=0), "large-wide": dict(merge_max_n=0, spec_wide_min=0),
         "large-aligned": dict(merge_max_n=0, split_align=16)}
PARAMS = list(itertools.product(CASES, sorted(PATHS)))


@pytest.fixture(scope="module", params=PARAMS,
                ids=["%s-L%d-m%s-%s" % (c + (p,)) for c, p in PARAMS])
def case(request):
    (name, levels, macro), path = request.param
    w = small_workload(name, levels, macro)
    w["coarse"] = min(w["coarse"], levels - 1)
    P = gpu_problem(w, outer="fgmres", **PATHS[path])
    yield w, P, path
    P.close()


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def _interior_special_colours(P, d, n):
    """Colours (i + j + k mod d + 1) that hold an interior interface vertex:
    under no-slip the velocity special launch of a colour covers only those
    rows (the boundary ones are fixed), and is made only if there are any."""
    cls = P.vertex_class()[0].reshape((n + 1,) * d)
    col = sum(np.indices(cls.shape)) % (d + 1)
    inner = ((cls & 1) != 0) & ((cls & 2) == 0)
    return {c for c in range(d + 1) if inner[col == c].any()}


def _check_large_launches(c, d, path, steps, form, colours):
    """Launch counts of `steps` smoothing steps on one level through the
    large-level kernels (every colour list holds boundary vertices, so every
    pressure special launch is made; velocity special launches are made for
    the colours in `colours`; the gradient and interface forms skip the
    repeated colour at the turn of the symmetric sweep)."""
    m = d + 1
    seq = list(range(m)) + list(range(m - 1 if form == "strain" else m - 2, -1, -1))
    vel = len(seq) * steps
    assert c["gs_vel_merged"] == c["p_rhs_merged"] == c["gs_p_merged"] == 0, c
    assert c["vel_rhs"] == steps and c["p_rhs_grouped"] == steps, c
    assert c["gs_vel_bulk"] == vel, c
    assert c["gs_vel_special"] == sum(k in colours for k in seq) * steps, (c, colours)
    assert c["gs_p_bulk"] == d * steps, c
    if path == "large-wide":
        assert c["gs_p_special_wide"] == m * steps and c["gs_p_special"] == 0, c
    else:
        assert c["gs_p_special"] == m * steps and c["gs_p_special_wide"] == 0, c


@pytest.mark.parametrize("block", ["velocity", "full"])
@pytest.mark.parametrize("form", ["gradient", "strain", "interface"])
def test_apply_and_residual_large_path(case, form, block):
    """Bulk rows of applies and residuals through the LDS-tiled kernel of
    the large 3D levels (2D keeps one vertex per thread): K x and b - K x
    against the assembled oracle operator, 1e-12 of max(|K| |x|)."""
    import torch
    from oracle import assemble
    from tests.gpu_common import abs_scale, assert_close_scaled
    w, P, path = case
    D = assemble.Discretisation(w["dim"], w["n"], w["inclusions"], w["mu"])
    K = D.stokes(form)
    N = D.N
    if block == "velocity":
        K = K[:w["dim"] * N][:, :w["dim"] * N]
    x = iss_inputs.random_vector(w["dim"], w["n"], seed=125)
    b = iss_inputs.random_rhs(w["dim"], w["n"], seed=126)
    if block == "full":
        b[w["dim"] * N:] = iss_inputs.random_vector(w["dim"], w["n"], seed=127)[w["dim"] * N:]
    xg, y = to_dev(x), torch.empty(x.size, dtype=torch.float64, device="cuda")
    P.launch_counts(reset=True)
    P.apply(form, xg, y, block=block)
    c = P.launch_counts()
    assert c["apply_tiled" if w["dim"] == 3 else "apply_bulk"] == 1, c
    nv = K.shape[0]
    ref = K @ x[:nv]
    scale = abs_scale(K, x[:nv])
    assert_close_scaled(to_host(y)[:nv], ref, scale, 1e-12, "%s/%s apply" % (form, block))
    if block == "full":
        r = torch.empty_like(y)
        P.residual(form, xg, to_dev(b), r)
        assert_close_scaled(to_host(r), b - K @ x, scale + np.abs(b), 1e-12, "%s residual" % form)


@pytest.mark.parametrize("form", ["gradient", "strain", "interface"])
def test_smoother_steps_large_path(case, form):
    w, P, path = case
    lv = mg.Level(w["dim"], w["n"], w["inclusions"], w["mu"], form)
    x = iss_inputs.random_vector(w["dim"], w["n"], seed=121)
    b = iss_inputs.random_rhs(w["dim"], w["n"], seed=122)
    xg = to_dev(x)
    P.launch_counts(reset=True)
    P.smooth(form, xg, to_dev(b), nsteps=2)
    _check_large_launches(P.launch_counts(), w["dim"], path, 2, form,
                          _interior_special_colours(P, w["dim"], w["n"]))
    ref = mg.smooth(lv, x, b, 2)
    assert _rel(to_host(xg), ref) < 1e-11, form


@pytest.mark.parametrize("form", ["strain", "interface"])
def test_smoother_step_fp32_large_path(case, form):
    import torch
    w, P, path = case
    lv = mg.Level(w["dim"], w["n"], w["inclusions"], w["mu"], form)
    x = iss_inputs.random_vector(w["dim"], w["n"], seed=123).astype(np.float32).astype(np.float64)
    b = iss_inputs.random_rhs(w["dim"], w["n"], seed=124).astype(np.float32).astype(np.float64)
    xg = to_dev(x, torch.float32)
    P.launch_counts(reset=True)
    P.smooth(form, xg, to_dev(b, torch.float32), nsteps=1)
    _check_large_launches(P.launch_counts(), w["dim"], path, 1, form,
                          _interior_special_colours(P, w["dim"], w["n"]))
    ref = mg.smooth(lv, x, b, 1)
    assert _rel(to_host(xg), ref) < 1e-5, form


@pytest.mark.parametrize("form", ["gradient", "strain", "interface"])
def test_vcycle_large_path(case, form):
    w, P, path = case
    H = mg.Hierarchy(w["dim"], w["macro"], w["levels"], w["coarse"], w["inclusions"], w["mu"], form)
    x = iss_inputs.random_vector(w["dim"], w["n"], seed=128)
    b = iss_inputs.random_rhs(w["dim"], w["n"], seed=129)
    xg = to_dev(x)
    P.launch_counts(reset=True)
    P.vcycle(form, xg, to_dev(b))
    c = P.launch_counts()
    assert c["gs_vel_bulk"] > 0 and c["gs_vel_merged"] == 0 and c["p_rhs_merged"] == 0, c
    ref = H.vcycle(w["levels"], x, b)
    assert _rel(to_host(xg), ref) < 1e-10, form


def test_vcycle_fp32_large_path(case):
    import torch
    w, P, path = case
    H = mg.Hierarchy(w["dim"], w["macro"], w["levels"], w["coarse"], w["inclusions"], w["mu"], "interface")
    x = iss_inputs.random_vector(w["dim"], w["n"], seed=130).astype(np.float32).astype(np.float64)
    b = iss_inputs.random_rhs(w["dim"], w["n"], seed=131).astype(np.float32).astype(np.float64)
    xg = to_dev(x, torch.float32)
    P.vcycle("interface", xg, to_dev(b, torch.float32))
    ref = H.vcycle(w["levels"], x, b)
    assert _rel(to_host(xg), ref) < 1e-4


@pytest.mark.parametrize("mid", [None, "strain"])
@pytest.mark.parametrize("name,levels", [("sphere_3d", 4), ("sinker_3d", 4)])
def test_vcycle_default_configuration_large_path(name, levels, mid):
    """The benchmark's V-cycle (averaged coarse viscosity, strain form on
    the coarsest level, optionally on every level below the finest, V(5,5),
    omega 0.6) through the large-level kernels on every level."""
    w = small_workload(name, levels)
    P = gpu_problem(w, coarse_mu="average", coarse_form="strain", mid_form=mid, omega=0.6, nu1=5, nu2=5,
                    merge_max_n=0, spec_wide_min=0)
    H = mg.Hierarchy(w["dim"], w["macro"], w["levels"], w["coarse"], w["inclusions"], w["mu"],
                     "interface", nu1=5, nu2=5, omega=0.6, coarse_mu="average", coarse_form="strain",
                     mid_form=mid)
    x = iss_inputs.random_vector(w["dim"], w["n"], seed=132)
    b = iss_inputs.random_rhs(w["dim"], w["n"], seed=133)
    xg = to_dev(x)
    P.vcycle("interface", xg, to_dev(b))
    ref = H.vcycle(w["levels"], x, b)
    assert _rel(to_host(xg), ref) < 1e-10
    P.close()


def test_default_path_is_merged_at_small_sizes():
    """Without the options, levels up to 65^3 take the merged launches."""
    w = small_workload("sphere_3d", 4)
    P = gpu_problem(w)
    x = to_dev(iss_inputs.random_vector(3, w["n"], seed=134))
    b = to_dev(iss_inputs.random_rhs(3, w["n"], seed=135))
    P.launch_counts(reset=True)
    P.smooth("interface", x, b, nsteps=1)
    c = P.launch_counts()
    assert c["gs_vel_merged"] == 7 and c["p_rhs_merged"] == 1 and c["gs_p_merged"] == 3, c
    assert c["gs_vel_bulk"] == c["p_rhs_grouped"] == c["gs_p_bulk"] == 0, c
    P.close()


def test_smoother_step_large_path_65():
    """One interface-form smoothing step on the 65^3 sinker through the
    large-level kernels.  Its special-row lists span 33 (velocity, interior
    rows) to 129 (pressure, one-wave groups) workgroups per colour, so the
    special-only kernels hand the XCDs permuted runs of 2 and 4 workgroups
    (the smaller cases above stay below the 16 workgroups from which the
    mapping permutes the velocity lists)."""
    w = small_workload("sinker_3d", 5)
    P = gpu_problem(w, merge_max_n=0)
    lv = mg.Level(3, w["n"], w["inclusions"], w["mu"], "interface")
    x = iss_inputs.random_vector(3, w["n"], seed=136)
    b = iss_inputs.random_rhs(3, w["n"], seed=137)
    xg = to_dev(x)
    P.launch_counts(reset=True)
    P.smooth("interface", xg, to_dev(b), nsteps=1)
    c = P.launch_counts()
    assert c["gs_vel_special"] == 7 and c["gs_p_special"] == 4 and c["gs_vel_merged"] == 0, c
    assert _rel(to_host(xg), mg.smooth(lv, x, b, 1)) < 1e-11
    P.close()
