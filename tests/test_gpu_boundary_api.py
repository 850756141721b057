"""The boundary calls around the hot path: a caller-owned workspace and a
problem posed by one viscosity phase per fine element.

* Workspace: a problem whose work buffers come from a bound device region
  gives the same bits as one that allocates them itself (smoothing,
  V-cycle, FGMRES solve, rate measurement); a region smaller than
  iss_workspace_bytes ends in ISS_E_NOWS; binding after the first use is
  rejected.
* Per-element phases: the phases an inclusion list produces, passed per
  element, give the same problem (vertex classes, applies bit for bit); an
  arbitrary per-element field (no geometry) matches the oracle assembled
  with the same element viscosities (applies 1e-12 of max |K||x|, one
  smoothing step 1e-11)."""
import numpy as np
import pytest

import iss_inputs
from oracle import assemble, mesh, multigrid as mg, problem as oprob
from tests.gpu_common import abs_scale, assert_close_scaled, gpu_problem, small_workload, to_dev, to_host

pytestmark = pytest.mark.gpu

PERMS = {3: [(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)], 2: [(0, 1), (1, 0)]}


def library_elements(dim, n):
    """Vertex ids of the lattice elements in the library's element order:
    cell c = ci + n (cj + n ck) (x fastest), then the Kuhn type, the axis
    order of the path from the cell's corner to its opposite corner."""
    out = []
    for c in range(n ** dim):
        corner = np.array([(c // n ** a) % n for a in range(dim)])
        for perm in PERMS[dim]:
            cur = corner.copy()
            v = [mesh.vertex_index(dim, n, cur)]
            for ax in perm:
                cur[ax] += 1
                v.append(mesh.vertex_index(dim, n, cur))
            out.append(v)
    return np.array(out, dtype=np.int64)


def test_workspace_gives_identical_results():
    import torch
    w = small_workload("sinker_3d", 4)
    kw = dict(outer="fgmres", coarse_mu="average", coarse_form="strain", mid_form="strain", restart=30,
              cycles=2, omega=0.6)
    b = to_dev(iss_inputs.random_rhs(3, w["n"], seed=140))
    x0 = to_dev(iss_inputs.random_vector(3, w["n"], seed=141))
    out = []
    for bound in (False, True):
        P = gpu_problem(w, **kw)
        if bound:
            nbytes = P.workspace_bytes("fp64")
            buf = torch.empty(nbytes // 8 + 32, dtype=torch.float64, device="cuda")
            off = (-buf.data_ptr()) % 256
            P.bind_workspace(buf.view(torch.uint8)[off:off + nbytes])
        xs = x0.clone()
        P.smooth("interface", xs, b, nsteps=2)
        xv = x0.clone()
        P.vcycle("interface", xv, b)
        xsol = torch.zeros_like(b)
        info = P.solve("interface", xsol, b, rtol=1e-8, maxit=40, raise_on_fail=False)
        xr = x0.clone()
        rates = P.asymptotic_rate("interface", xr, iters=5)
        out.append((xs, xv, xsol, info["history"], rates))
        if bound:
            # binding again after use is rejected
            from paper_1604_07994_amd.binding import IssError
            with pytest.raises(IssError):
                P.bind_workspace(buf.view(torch.uint8)[off:off + nbytes])
        P.close()
    (a, b_) = out
    for u, v in zip(a[:3], b_[:3]):
        assert torch.equal(u, v)
    assert a[3] == b_[3] and a[4] == b_[4]


def test_workspace_too_small_is_reported():
    import ctypes
    import torch
    from paper_1604_07994_amd import binding
    w = small_workload("sphere_3d", 4)
    P = gpu_problem(w, outer="fgmres", restart=20)
    nbytes = P.workspace_bytes("fp64")
    buf = torch.empty(nbytes // 16, dtype=torch.float64, device="cuda")
    off = (-buf.data_ptr()) % 256
    P.bind_workspace(buf.view(torch.uint8)[off:off + nbytes // 2])
    b = to_dev(iss_inputs.random_rhs(3, w["n"], seed=142))
    x = torch.zeros_like(b)
    L = binding.lib()
    info = binding.SolveInfo()
    rc = L.iss_solve(P._h, 2, 0, 1e-8, 50, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(b.data_ptr()),
                     ctypes.byref(info), binding._stream())
    assert rc == -6 and b"workspace too small" in L.iss_last_error()
    P.close()


def test_element_phases_equal_inclusions():
    import torch
    from paper_1604_07994_amd import Problem
    w = small_workload("sinker_3d", 4)
    n = w["n"]
    E = library_elements(3, n)
    ph = oprob.element_phase(3, n, E, w["inclusions"]).astype(np.uint8)
    Pi = gpu_problem(w, coarse_mu="average")
    Pe = Problem.from_elems(3, w["macro"], w["levels"], w["coarse"], ph, w["mu"])
    ci, ni, bi = Pi.vertex_class()
    ce, ne, be = Pe.vertex_class()
    assert np.array_equal(ci, ce) and ni == ne and bi == be
    x = to_dev(iss_inputs.random_vector(3, n, seed=143))
    for form in ("strain", "interface"):
        yi, ye = torch.empty_like(x), torch.empty_like(x)
        Pi.apply(form, x, yi)
        Pe.apply(form, x, ye)
        assert torch.equal(yi, ye), form
    b = to_dev(iss_inputs.random_rhs(3, n, seed=144))
    xi, xe = x.clone(), x.clone()
    Pi.vcycle("interface", xi, b)
    Pe.vcycle("interface", xe, b)
    assert torch.equal(xi, xe)
    Pi.close()
    Pe.close()


@pytest.mark.parametrize("dim,levels,macro", [(3, 3, 2), (2, 5, 1)])
def test_arbitrary_element_field_matches_oracle(dim, levels, macro):
    """Three phases drawn at random per element (mu 1, 30, 900): almost every
    vertex is an interface vertex.  The oracle assembles K from the same
    element viscosities (its own element order, matched by vertex sets)."""
    import torch
    from paper_1604_07994_amd import Problem
    n = macro * 2 ** levels
    mu = [1.0, 30.0, 900.0]
    E = library_elements(dim, n)
    ph = np.random.default_rng(145).integers(0, 3, len(E)).astype(np.uint8)
    P = Problem.from_elems(dim, macro, levels, max(1, levels - 1), ph, mu)
    Eo = mesh.kuhn_elements(dim, n)
    pos = {tuple(sorted(e)): i for i, e in enumerate(E)}
    mu_e = np.array([mu[ph[pos[tuple(sorted(e))]]] for e in Eo])
    D = assemble.Discretisation(dim, n, [], mu, mu_e=mu_e)
    x = iss_inputs.random_vector(dim, n, seed=146)
    xg = to_dev(x)
    for form in ("gradient", "strain", "interface"):
        K = D.stokes(form)
        y = torch.empty_like(xg)
        P.apply(form, xg, y)
        assert_close_scaled(to_host(y), K @ x, abs_scale(K, x), 1e-12, "%dD %s" % (dim, form))
    b = iss_inputs.random_rhs(dim, n, seed=147)
    lv = mg.Level(dim, n, [], mu, "interface", mu_e=mu_e)
    xs = to_dev(x)
    P.smooth("interface", xs, to_dev(b), nsteps=1)
    ref = mg.smooth(lv, x, b, 1)
    assert np.abs(to_host(xs) - ref).max() <= 1e-11 * np.abs(ref).max()
    P.close()
