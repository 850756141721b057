"""Pins of the oracle's free-slip boundary condition (eq. boundary), the
box inclusions of the viscosity-columns problem (Sec. 4) and the nodal
force load, against closed forms and identities (no GPU)."""
import numpy as np
import pytest
import scipy.sparse as sp
import sympy as sy

import iss_inputs
from oracle import assemble, fem, mesh, multigrid as mg, problem

COLUMNS = iss_inputs.workload('columns_3d')['inclusions']


# --- fixed set --------------------------------------------------------------

@pytest.mark.parametrize("dim", [2, 3])
def test_fixed_sets_by_brute_force(dim):
    """No-slip fixes every component of a boundary vertex; free-slip fixes
    u . n on each face, i.e. component k exactly on the faces x_k = 0, 1
    (an edge or corner vertex has every normal of its faces fixed)."""
    n = 4
    ijk = mesh.vertex_ijk(dim, n)
    fs = mesh.fixed_velocity(dim, n, 'freeslip')
    ns = mesh.fixed_velocity(dim, n, 'noslip')
    for v in range(len(ijk)):
        faces = [a for a in range(dim) if ijk[v, a] in (0, n)]
        for k in range(dim):
            assert fs[k, v] == (k in faces)
            assert ns[k, v] == bool(faces)
    assert fs.sum() == dim * 2 * (n + 1) ** (dim - 1)


# --- the manufactured free-slip flow ------------------------------------------

def _fs_flow():
    """u = (sin pi x cos pi y, -cos pi x sin pi y[, 0]), p = cos pi x cos pi y;
    constant mu."""
    x, y, z = sy.symbols('x y z', real=True)
    u = [sy.sin(sy.pi * x) * sy.cos(sy.pi * y), -sy.cos(sy.pi * x) * sy.sin(sy.pi * y), sy.Integer(0)]
    p = sy.cos(sy.pi * x) * sy.cos(sy.pi * y)
    return (x, y, z), u, p


def test_freeslip_flow_satisfies_the_boundary_conditions():
    """The manufactured flow is solenoidal, has u . n = 0 and zero tangential
    traction n x sigma n = 0 on every face of the unit cube (eq. boundary,
    free-slip): the test problem below has a known solution."""
    X, u, p = _fs_flow()
    assert sy.simplify(sum(sy.diff(u[a], X[a]) for a in range(3))) == 0
    for a in range(3):
        for side in (0, 1):
            assert sy.simplify(u[a].subs(X[a], side)) == 0
            for t in range(3):
                if t == a:
                    continue
                shear = sy.diff(u[a], X[t]) + sy.diff(u[t], X[a])
                assert sy.simplify(shear.subs(X[a], side)) == 0


def _fs_errors(dim, n, form, bc, mu=3.0):
    X, u, p = _fs_flow()
    f = [sy.lambdify(X, -mu * sum(sy.diff(u[a], X[b], 2) for b in range(3)) + sy.diff(p, X[a]), 'numpy')
         for a in range(dim)]
    ue = [sy.lambdify(X, u[a], 'numpy') for a in range(dim)]
    D = assemble.Discretisation(dim, n, [], [mu], bc=bc)
    C = mesh.vertex_coords(dim, n)
    Cz = np.concatenate([C, np.zeros((len(C), 3 - dim))], axis=1)
    fn = np.stack([np.broadcast_to(np.asarray(fa(*Cz.T), dtype=np.float64), (len(C),)) for fa in f], axis=1)
    b = problem.rhs_from_nodal_force(dim, n, D.elems, fn) * D.free_mask()
    lv = mg.Level(dim, n, [], [mu], form, bc=bc)
    xh = mg.direct_solve(lv, b)
    M = D.mass()
    err = 0.0
    for a in range(dim):
        e = xh[a * D.N:(a + 1) * D.N] - np.broadcast_to(np.asarray(ue[a](*Cz.T), dtype=np.float64), (D.N,))
        err += e @ (M @ e)
    return np.sqrt(err)


@pytest.mark.parametrize("form", ["strain", "interface", "gradient"])
def test_freeslip_flow_converges_at_second_order_2d(form):
    """O(h^2) L2 convergence to the free-slip flow in every form (for
    constant mu and this flow all three are consistent); the same problem
    posed with no-slip does not converge (its tangential boundary velocity
    is wrong), so a dropped or misplaced free component fails here."""
    errs = [_fs_errors(2, n, form, 'freeslip') for n in (8, 16, 32, 64)]
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert rates[-1] >= 1.8 and rates[-2] >= 1.7, (form, errs, rates)
    wrong = [_fs_errors(2, n, form, 'noslip') for n in (16, 32)]
    assert wrong[1] > 0.5 * wrong[0] and wrong[1] > 20 * errs[2], (wrong, errs)


def test_freeslip_flow_converges_3d():
    errs = [_fs_errors(3, n, 'interface', 'freeslip') for n in (4, 8)]
    assert np.log2(errs[0] / errs[1]) >= 1.5, errs


@pytest.mark.parametrize("dim", [2, 3])
def test_boundary_rows_on_gamma_f(dim):
    """Sec. 2.2: with one viscosity the Laplacian rows equal the a_tr rows at
    interior vertices; on Gamma_F the cross terms leave a boundary integral
    of u_i times tangential derivatives of the test function.  Without
    fixed components (a traction-free boundary) it is non-zero, so the
    gradient form differs from a_tr exactly on boundary rows and the full
    rows are needed there.  Under free-slip on the cube's planar faces the
    normal component, the only one that meets the face's normal in that
    integral, vanishes on the whole face, so the three operators coincide;
    the interface form (full rows on the boundary) equals a_tr either way."""
    n = 4
    D = assemble.Discretisation(dim, n, [], [2.5], bc='freeslip')
    Kt = D.stokes('tr')
    for form in ('interface', 'gradient'):
        assert abs(D.stokes(form) - Kt).max() < 1e-13 * abs(Kt).max(), form
    At = D.viscous('tr')
    Ag = D.viscous('gradient')
    Ai = D.viscous('interface')
    assert abs(Ai - At).max() < 1e-13 * abs(At).max()
    diff = abs(Ag - At).tocsr()
    rows = np.nonzero(np.asarray(diff.max(axis=1).todense()).ravel() > 1e-12)[0]
    assert len(rows) > 0 and np.all(D.boundary[rows % D.N])


def test_freeslip_hierarchy_one_level_is_direct():
    """A V-cycle whose finest level is the coarsest is the direct solve:
    the free-slip fixed set reaches the coarse solver's free dofs."""
    H = mg.Hierarchy(3, 2, 1, 1, COLUMNS, [1.0, 10.0], 'interface', bc='freeslip')
    lv = H.levels[1]
    b = iss_inputs.random_rhs(3, 4, seed=3, bc='freeslip')
    x = H.vcycle(1, np.zeros_like(b), b)
    assert np.linalg.norm(lv.K @ x - b) < 1e-11 * np.linalg.norm(b)


def test_freeslip_multigrid_contracts():
    """Two-grid V(3,3) on the columns problem with free-slip contracts at a
    rate of the order of the paper's (Sec. 5 reports about 0.24-0.30)."""
    H = mg.Hierarchy(3, 2, 2, 1, COLUMNS, [1.0, 10.0], 'interface', bc='freeslip', coarse_mu='average',
                     coarse_form='strain')
    rho = H.asymptotic_rate(iters=30, seed=1)
    assert rho < 0.5, rho


def test_coarse_swap_needs_the_rhs_modification():
    """Sec. 5: replacing a_tr by a_sym on the coarse grid naively degrades
    the multigrid; the momentum right-hand side r_1 + B^T M^-1 r_2 (the
    paper's r_1 - B^T M^-1 r_2 with its opposite sign of B) recovers part
    of it.  Two-grid V(3,3)+2, omega 0.3, on the columns problem (17^3 over
    9^3): rate(same form) < rate(modified swap) < rate(naive swap) for the
    interface and the gradient form, and the strain form is unaffected."""
    w = iss_inputs.workload('columns_3d')

    def rate(form, **kw):
        H = mg.Hierarchy(3, 4, 2, 1, w['inclusions'], w['mu'], form, nu1=3, nu2=3, nu_inc=2, omega=0.3,
                         coarse_mu='average', bc='freeslip', **kw)
        return H.asymptotic_rate(iters=40, seed=1)

    for form in ('interface', 'gradient'):
        same = rate(form)
        mod = rate(form, coarse_form='strain', coarse_rhs_mod=True)
        naive = rate(form, coarse_form='strain')
        assert same < mod < naive, (form, same, mod, naive)
    s0 = rate('strain')
    assert abs(rate('strain', coarse_form='strain', coarse_rhs_mod=True) - s0) < 1e-12


# --- columns geometry and the force load ---------------------------------------

@pytest.mark.parametrize("n", [4, 8])
def test_columns_are_resolved_boxes(n):
    """The columns (0, 1/4)^2 x (0, 1) and (3/4, 1)^2 x (0, 1) fill 1/8 of the
    cube and are resolved by every lattice with n divisible by 4: exactly
    n^3 6 / 8 elements take the column phase, and interface vertices lie on
    the column walls x or y in {1/4, 3/4} only."""
    E = mesh.kuhn_elements(3, n)
    ph = problem.element_phase(3, n, E, COLUMNS)
    assert ph.sum() == n ** 3 * 6 // 8
    mu_e = np.array([1.0, 10.0])[ph]
    itf = problem.interface_vertices(3, n, E, mu_e)
    X = mesh.vertex_coords(3, n)[itf]
    on_wall = np.isclose(X[:, 0], 0.25) | np.isclose(X[:, 0], 0.75) | np.isclose(X[:, 1], 0.25) | \
        np.isclose(X[:, 1], 0.75)
    assert itf.sum() > 0 and np.all(on_wall)


@pytest.mark.parametrize("dim", [2, 3])
def test_nodal_force_load_integrates_linear_fields(dim):
    """b = M f integrates P1 fields exactly: sum_j (M f)_j = int f, here for
    f = 1 (volume 1) and f = x_a (1/2); a permuted element list gives the
    same load (assembly order does not matter)."""
    n = 4
    E = mesh.kuhn_elements(dim, n)
    X = mesh.vertex_coords(dim, n)
    N = len(X)
    for a in range(dim):
        f = np.zeros((N, dim))
        f[:, a] = 1.0
        b = problem.rhs_from_nodal_force(dim, n, E, f)
        assert abs(b[a * N:(a + 1) * N].sum() - 1.0) < 1e-13
        f[:, a] = X[:, a]
        b = problem.rhs_from_nodal_force(dim, n, E, f)
        assert abs(b[a * N:(a + 1) * N].sum() - 0.5) < 1e-13
        b2 = problem.rhs_from_nodal_force(dim, n, E[::-1], f)
        assert np.allclose(b, b2, rtol=0, atol=1e-15)
        assert np.all(b[dim * N:] == 0)


def test_column_force_closed_form():
    """The nodal force of the columns problem: only the last component is
    non-zero, -cos(2 pi x) cos(2 pi y) sin(pi z), zero on z = 0 and z = 1."""
    n = 8
    f = iss_inputs.column_force(3, n)
    X = mesh.vertex_coords(3, n)
    assert np.all(f[:2] == 0)
    ref = -np.cos(2 * np.pi * X[:, 0]) * np.cos(2 * np.pi * X[:, 1]) * np.sin(np.pi * X[:, 2])
    assert np.allclose(f[2], ref, atol=1e-15)
    assert np.allclose(f[2][np.isclose(X[:, 2], 0.0) | np.isclose(X[:, 2], 1.0)], 0.0, atol=1e-15)
