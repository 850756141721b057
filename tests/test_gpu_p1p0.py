"""GPU parity of the stabilised P1-P0 operator of Sec. 3 (P0 pressure on the
elements, the interior-penalty form of eq. stabc, the local flux
post-process) against the oracle's assembled P1-P0 system (oracle.p1p0).

Tolerances: K x within 1e-12 of max(|K| |x|) (FP64, sums of at most 15
velocity-block terms, 24 B0^T terms and 4 + d facet terms per row); fluxes
within 1e-13 of max |flux|; on the oracle's discrete Couette solution the
GPU fluxes of every element sum to zero within 1e-12 of the largest flux
(Sec. 3: exact element-wise mass balance)."""
import numpy as np
import pytest

import iss_inputs
from oracle import p1p0
from tests.gpu_common import abs_scale, assert_close_scaled, gpu_problem, small_workload, to_dev, to_host

pytestmark = pytest.mark.gpu

CASES = [("sphere_3d", 2, None, "noslip"), ("columns_3d", 1, 4, "freeslip"), ("sinker_3d", 2, 2, "noslip"),
         ("square_split_2d", 3, None, "noslip"), ("square_split_2d", 4, None, "freeslip")]


def _case(name, levels, macro, bc):
    w = small_workload(name, levels, macro)
    w["coarse"] = 1
    w["bc"] = bc
    return w


@pytest.mark.parametrize("gamma", [1.0, 0.4])
@pytest.mark.parametrize("form", ["gradient", "strain", "interface"])
@pytest.mark.parametrize("case", CASES, ids=["%s-L%d-m%s-%s" % c for c in CASES])
def test_p1p0_apply_matches_oracle(case, form, gamma):
    import torch
    w = _case(*case)
    d, n = w["dim"], w["n"]
    P = gpu_problem(w)
    O = p1p0.P1P0(d, n, w["inclusions"], w["mu"], gamma=gamma, bc=w["bc"])
    assert P.num_elements() == O.ne
    rng = np.random.default_rng(170)
    x = rng.uniform(-1, 1, O.ndof) * O.free_mask()
    K = O.stokes(form)
    xg = to_dev(x)
    y = torch.empty_like(xg)
    P.p1p0_apply(form, xg, y, gamma=gamma)
    assert_close_scaled(to_host(y), K @ x, abs_scale(K, x), 1e-12, "%s P1-P0 apply" % form)
    P.close()


@pytest.mark.parametrize("case", CASES, ids=["%s-L%d-m%s-%s" % c for c in CASES])
def test_p1p0_flux_matches_oracle(case):
    import torch
    w = _case(*case)
    d, n = w["dim"], w["n"]
    P = gpu_problem(w)
    O = p1p0.P1P0(d, n, w["inclusions"], w["mu"], gamma=0.8, bc=w["bc"])
    x = np.random.default_rng(171).uniform(-1, 1, O.ndof)
    ref = O.fluxes(x)
    fl = torch.empty(O.ne * (d + 1), dtype=torch.float64, device="cuda")
    P.p1p0_flux(to_dev(x), fl, gamma=0.8)
    got = to_host(fl).reshape(O.ne, d + 1)
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()
    P.close()


@pytest.mark.parametrize("level", [0, 1])
def test_couette_fluxes_balance_on_the_gpu(level):
    """The oracle's discrete Couette solution (Sec. 4; mu1 / mu2 = 10^3,
    gamma = 1, Dirichlet data of the exact solution): the GPU post-processed
    fluxes of every element sum to zero, and the GPU P1-P0 apply reproduces
    the pressure rows B0 u - C p = 0 of the discrete system."""
    import torch
    from paper_1604_07994_amd import Problem
    O, x, _ = p1p0.couette_problem(level)
    n = O.n
    inc = [{'kind': 'halfspace', 'axis': 1, 'threshold': 0.5, 'phase': 1}]
    P = Problem(3, n // 2, 1, 1, inc, [1e-3, 1.0])       # n = (n / 2) 2^1 cells per axis
    fl = torch.empty(O.ne * 4, dtype=torch.float64, device="cuda")
    P.p1p0_flux(to_dev(x), fl)
    f = to_host(fl).reshape(O.ne, 4)
    assert np.abs(f.sum(axis=1)).max() <= 1e-12 * np.abs(f).max()
    # pressure rows of K x (the velocity rows of the library are masked on
    # the Dirichlet dofs, which carry the boundary data here)
    y = torch.empty(O.ndof, dtype=torch.float64, device="cuda")
    P.p1p0_apply("interface", to_dev(x), y)
    yp = to_host(y)[3 * O.N:]
    B = O.divergence()
    scale = np.abs(B) @ np.abs(x[:3 * O.N])
    assert np.abs(yp).max() <= 1e-12 * scale.max()
    P.close()


def test_p1p0_with_per_element_phases():
    """A problem posed by one phase per element (random three-phase field):
    the P1-P0 apply uses those element phases for the penalty facets."""
    import torch
    from paper_1604_07994_amd import Problem
    from tests.test_gpu_boundary_api import library_elements
    n, mu = 4, [1.0, 30.0, 900.0]
    E = library_elements(3, n)
    ph = np.random.default_rng(172).integers(0, 3, len(E)).astype(np.uint8)
    P = Problem.from_elems(3, 2, 1, 1, ph, mu)
    O = p1p0.P1P0(3, n, [], mu, mu_e=np.array(mu)[ph])
    assert np.array_equal(mesh_elements_sorted(E), mesh_elements_sorted(O.E))
    x = np.random.default_rng(173).uniform(-1, 1, O.ndof) * O.free_mask()
    K = O.stokes("interface")
    xg = to_dev(x)
    y = torch.empty_like(xg)
    P.p1p0_apply("interface", xg, y)
    assert_close_scaled(to_host(y), K @ x, abs_scale(K, x), 1e-12, "P1-P0 apply, element phases")
    P.close()


def mesh_elements_sorted(E):
    return np.sort(np.asarray(E), axis=1)


@pytest.mark.parametrize("case", [("sphere_3d", 4, None, "noslip"), ("columns_3d", 2, 4, "freeslip")],
                         ids=["sphere_3d-L4-noslip", "columns_3d-L2-m4-freeslip"])
@pytest.mark.parametrize("form", ["interface", "strain"])
def test_p1p0_apply_through_the_tiled_velocity_apply(case, form):
    """The velocity part of the P1-P0 apply through the LDS-tiled z-march of
    the large levels (merge_max_n = 0; 17^3, two z chunks), as at 257^3."""
    import torch
    w = _case(*case)
    d, n = w["dim"], w["n"]
    P = gpu_problem(w, merge_max_n=0)
    O = p1p0.P1P0(d, n, w["inclusions"], w["mu"], gamma=1.0, bc=w["bc"])
    x = np.random.default_rng(174).uniform(-1, 1, O.ndof) * O.free_mask()
    K = O.stokes(form)
    y = torch.empty(O.ndof, dtype=torch.float64, device="cuda")
    P.p1p0_apply(form, to_dev(x), y, gamma=1.0)
    assert_close_scaled(to_host(y), K @ x, abs_scale(K, x), 1e-12, "%s P1-P0 apply, tiled" % form)
    P.close()
