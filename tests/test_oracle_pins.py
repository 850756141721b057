"""Pins of the CPU oracle against facts fixed by the paper and by the
mathematics (no GPU).  Each test names the passage or identity it checks."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla
import sympy as sy

import iss_inputs
from oracle import assemble, fem, manufactured, mesh, multigrid as mg, problem

SPHERE = [{'kind': 'sphere', 'center': (0.5, 0.5, 0.5), 'radius': 0.3, 'phase': 1}]
SPLIT = [{'kind': 'halfspace', 'axis': 0, 'threshold': 0.5, 'phase': 1}]


def disc(dim, n, contrast=100.0):
    inc = SPLIT if dim == 2 else SPHERE
    return assemble.Discretisation(dim, n, inc, [1.0, contrast])


def field(D, fn):
    """Nodal interpolant of a vector field fn(x) -> (N, d), field-major."""
    X = mesh.vertex_coords(D.dim, D.n)
    return fn(X).T.ravel()


# --- mesh -------------------------------------------------------------------

@pytest.mark.parametrize("dim,levels", [(2, 3), (3, 2)])
def test_bey_refinement_gives_kuhn_lattice(dim, levels):
    """Sec. 3 remark on Bey-refined meshes: refining the Kuhn split of the
    cube with Bey's rule gives exactly the Kuhn lattice elements."""
    c, e = mesh.macro_mesh(dim, 1)
    for _ in range(levels):
        c, e = mesh.bey_refine(c, e)
    n = 2 ** levels
    vid = mesh.vertex_index(dim, n, np.rint(c * n).astype(np.int64))
    got = {tuple(sorted(t)) for t in vid[e]}
    ref = {tuple(sorted(t)) for t in mesh.kuhn_elements(dim, n)}
    assert got == ref
    # volumes of the children are equal (uniform refinement)
    _, vol = fem.simplex_geometry(c[e])
    assert np.allclose(vol, vol[0])


def test_element_counts_and_incidence():
    for dim, per in ((2, 6), (3, 24)):
        n = 4
        E = mesh.kuhn_elements(dim, n)
        assert len(E) == n ** dim * (2 if dim == 2 else 6)
        cnt = np.bincount(E.ravel(), minlength=mesh.num_vertices(dim, n))
        inner = ~mesh.boundary_mask(dim, n)
        assert np.all(cnt[inner] == per)


# --- element matrices / assembly ------------------------------------------

@pytest.mark.parametrize("dim", [2, 3])
def test_laplacian_stencil_closed_form(dim):
    """Isoviscous rows are the Laplacian stencil (Sec. 2.2): on the Kuhn
    lattice mu h^{d-2} [2d at the centre, -1 at the 2d axis neighbours],
    zero weight on the diagonal directions."""
    n, mu = 6, 7.0
    D = assemble.Discretisation(dim, n, [], [mu])
    A = D.viscous('gradient').tocsr()
    v = int(mesh.vertex_index(dim, n, np.array([3] * dim)))
    ijk = mesh.vertex_ijk(dim, n)
    for k in range(dim):
        row = A.getrow(k * D.N + v)
        cols = row.indices[np.abs(row.data) > 1e-13]
        vals = row.toarray().ravel()
        assert np.all(cols // D.N == k)
        scale = mu * D.h ** (dim - 2)
        assert np.isclose(vals[k * D.N + v], 2 * dim * scale)
        for c in cols:
            off = ijk[c % D.N] - 3
            if np.abs(off).sum() == 1:
                assert np.isclose(vals[c], -scale)
            else:
                assert np.all(off == 0)


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("form", ["gradient", "strain", "tr", "interface"])
def test_symmetry_and_constants(dim, form):
    """All forms are symmetric (eq. newbil is symmetric) and annihilate
    constant velocity fields."""
    D = disc(dim, 6)
    A = D.viscous(form)
    if form != 'interface':
        assert abs(A - A.T).max() <= 1e-13 * abs(A).max()
    one = np.ones(dim * D.N)
    assert np.abs(A @ one).max() <= 1e-12 * abs(A).max()


@pytest.mark.parametrize("dim", [2, 3])
def test_interface_form_equals_tr_entrywise(dim):
    """Eq. equivalence-stencil: Laplacian rows away from the interface and
    a_tr rows on it give exactly the a_tr matrix (on the free dofs)."""
    for contrast in (10.0, 1e4):
        D = disc(dim, 8, contrast)
        A_if = D.velocity_operator('interface')
        A_tr = D.velocity_operator('tr')
        A_lap = D.velocity_operator('gradient')
        scale = abs(A_tr).max()
        assert abs(A_if - A_tr).max() <= 1e-13 * scale
        # and the gradient form differs, only on interface rows
        diff = abs(A_lap - A_tr).max(axis=1).toarray().ravel()
        rows_if = np.tile(D.interface & ~D.boundary, dim)
        assert diff[~rows_if].max() <= 1e-13 * scale
        assert diff[rows_if].max() > 1e-3 * scale


def test_rigid_rotation_and_trace_free_linear_fields():
    """a_sym and a_tr vanish on rigid rotations; a_tr = a_sym on solenoidal
    fields (Sec. 2: 'For solenoidal elements ... equal'); the gradient form
    does not (it is inconsistent, Sec. 1) -- but only on interface rows."""
    D = disc(3, 8, 50.0)
    rot = field(D, lambda X: np.stack([-X[:, 1], X[:, 0], 0 * X[:, 0]], 1))
    tfl = field(D, lambda X: np.stack([X[:, 0], -X[:, 1], 0 * X[:, 0]], 1))
    A = {f: D.viscous(f) for f in ('strain', 'tr', 'gradient')}
    s = abs(A['strain']).max()
    # full operators (no boundary conditions): pointwise sym grad = 0
    assert np.abs(A['strain'] @ rot).max() <= 1e-12 * s
    assert np.abs(A['tr'] @ rot).max() <= 1e-12 * s
    assert np.abs(A['tr'] @ tfl - A['strain'] @ tfl).max() <= 1e-12 * s
    inner = np.tile(~D.boundary, 3)
    rows_if = np.tile(D.interface, 3) & inner
    rows_iso = ~np.tile(D.interface, 3) & inner
    for u in (rot, tfl):
        y = A['gradient'] @ u
        assert np.abs(y[rows_iso]).max() <= 1e-12 * s
        assert np.abs(y[rows_if] - (A['strain'] @ u)[rows_if]).max() > 1e-3 * s
        assert np.abs((A['strain'] @ u)[rows_iso]).max() <= 1e-12 * s


@pytest.mark.parametrize("dim,expected", [(2, 0.0), (3, -3.0)])
def test_identity_field_energy(dim, expected):
    """Sec. 3: for v = x, a_dev(v, v) = 0 and a_tr(v, v) =
    -3 (mu_1 |Omega_1| + mu_2 |Omega_2|) in 3D (0 in 2D): a_tr is not
    positive semi-definite.  Full operator, no boundary conditions."""
    D = disc(dim, 6, 20.0)
    x = field(D, lambda X: X)
    e = x @ (D.viscous('tr') @ x)
    ref = expected * np.sum(D.mu_e * D.vol)
    assert np.isclose(e, ref, rtol=1e-12, atol=1e-12)
    # a_dev = a_tr + (1 - 2/d) (mu div, div) vanishes on v = x
    a_dev = D.viscous('tr') + (1 - 2.0 / dim) * D._coo(
        fem.viscous_element_matrices(D.G, D.vol, D.mu_e, 'div'),
        D._velocity_dofs(), D._velocity_dofs(), (dim * D.N, dim * D.N))
    assert abs(x @ (a_dev @ x)) <= 1e-11 * abs(ref if ref else 1.0)


@pytest.mark.parametrize("dim", [2, 3])
def test_divergence_and_gradient_on_linear_fields(dim):
    """b(v, q) = -(div v, q) (eq. weaks): for linear u, (B u)_j =
    -div(u) int lambda_j; for linear p and interior j, (B^T p)_(j,l) =
    d_l p int lambda_j.  int lambda_j is taken from the mass matrix row
    sums (an independent element routine)."""
    D = disc(dim, 6)
    B = D.divergence()
    lumped = np.asarray(D.mass().sum(axis=1)).ravel()
    coef = np.arange(1, dim * dim + 1, dtype=float).reshape(dim, dim) / 3.0
    u = field(D, lambda X: X @ coef.T)
    div = np.trace(coef)
    assert np.allclose(B @ u, -div * lumped, rtol=1e-12, atol=1e-14)
    g = np.arange(1, dim + 1) * 0.7
    p = mesh.vertex_coords(dim, D.n) @ g
    y = (B.T @ p).reshape(dim, D.N)
    inner = ~D.boundary
    for l in range(dim):
        assert np.allclose(y[l][inner], g[l] * lumped[inner], rtol=1e-12, atol=1e-14)
    # the centre weight of B is zero
    v = int(mesh.vertex_index(dim, D.n, np.array([3] * dim)))
    for k in range(dim):
        assert abs(B[v, k * D.N + v]) < 1e-15


def test_divergence_sums_to_zero_on_V_h():
    """int div u = 0 for u with zero boundary values: sum_j (B u)_j = 0."""
    D = disc(3, 6)
    u = iss_inputs.random_vector(3, 6, seed=1)[:3 * D.N]
    assert abs(np.sum(D.divergence() @ u)) < 1e-13


def test_stabilisation_closed_form():
    """C 1 = 0; isoviscous rows are beta h^2/mu times the Laplacian stencil
    (stabilised P1-P1 reading, beta = 1/12)."""
    n, mu = 6, 4.0
    D = assemble.Discretisation(3, n, [], [mu])
    C = D.stabilisation()
    assert np.abs(C @ np.ones(D.N)).max() < 1e-15
    v = int(mesh.vertex_index(3, n, np.array([2, 3, 4])))
    row = C.getrow(v).toarray().ravel()
    s = fem.STAB_BETA * D.h ** 2 / mu * D.h
    assert np.isclose(row[v], 6 * s)
    assert np.isclose(row[v + 1], -s) and np.isclose(row[v - (n + 1) ** 2], -s)
    assert abs(row[v + 1 + (n + 1)]) < 1e-16


def test_nullity_is_constant_pressure():
    """K = [[A, B^T], [B, -C]] (Sec. 5) restricted to free dofs has exactly
    one zero eigenvalue: the constant pressure (Sec. 1: uniqueness up to a
    constant, fixed by Q)."""
    for form in ('interface', 'strain'):
        D = assemble.Discretisation(3, 4, SPHERE, [1.0, 1e4])
        K = D.stokes(form)
        f = D.free_mask()
        Kf = K[f][:, f].toarray()
        s = 1.0 / np.sqrt(np.abs(np.diag(Kf)))      # Jacobi scaling
        w, V = np.linalg.eigh(s[:, None] * Kf * s[None, :])
        a = np.sort(np.abs(w))
        assert a[0] < 1e-12 * a[-1]
        assert a[1] > 1e-5 * a[-1]
        # the null vector is the constant pressure
        z = V[:, np.argmin(np.abs(w))] * s
        nv = z[-D.N:]
        assert np.abs(z[:-D.N]).max() < 1e-8 * np.abs(nv).max()
        assert np.ptp(nv) < 1e-8 * np.abs(nv).max()


@pytest.mark.parametrize("form", ["gradient", "strain", "interface"])
def test_colouring_has_no_same_colour_coupling(form):
    """The multicolour ordering (i+j+k) mod 4 (3D) never couples two distinct
    vertices of one colour, for every block of K."""
    D = disc(3, 6, 1e3)
    col = mg.colours(3, 6)
    K = D.stokes(form).tocoo()
    vi, vj = K.row % D.N, K.col % D.N
    bad = (vi != vj) & (col[vi] == col[vj]) & (np.abs(K.data) > 0)
    assert not bad.any()
    D2 = disc(2, 6, 1e3)
    K2 = D2.stokes(form).tocoo()
    c2 = mg.colours(2, 6)
    vi, vj = K2.row % D2.N, K2.col % D2.N
    assert not ((vi != vj) & (c2[vi] == c2[vj]) & (np.abs(K2.data) > 0)).any()


def test_every_colour_neighbours_every_other():
    """In 3D every interior vertex is coupled through the velocity block to
    vertices of all three other colours, so one colour phase of the smoother
    reads every colour of u (the bytes a single phase must move)."""
    D = disc(3, 6, 1e3)
    col = mg.colours(3, 6)
    interior = np.flatnonzero(~D.boundary)
    for form in ("interface", "strain"):
        A = D.stokes(form).tocsr()[:D.N, :D.N]
        for v in interior:
            lo, hi = A.indptr[v], A.indptr[v + 1]
            nb = A.indices[lo:hi][(A.indices[lo:hi] != v) & (A.data[lo:hi] != 0)]
            assert set(((col[nb] - col[v]) % 4).tolist()) == {1, 2, 3}, (form, v)


def _point_gs(lv, x, b, groups):
    """Point-block Gauss-Seidel on the velocity block: every vertex of each
    group in turn solves its d x d block for its residual (fixed velocity
    entries stay)."""
    A, N, d = lv.A.tocsr(), lv.N, lv.dim
    free = lv.free[:d * N].reshape(d, N)
    for verts in groups:
        for v in verts:
            idx = np.array([v + k * N for k in range(d) if free[k, v]])
            if len(idx) == 0:
                continue
            r = b[idx] - A[idx] @ x
            x[idx] += np.linalg.solve(A[idx][:, idx].toarray(), r)
    return x


@pytest.mark.parametrize("form", ["interface", "strain"])
def test_z_wavefront_colour_order_equals_the_colour_sweep(form):
    """A forward colour sweep (colour 0 everywhere, then 1, 2, 3) gives the
    same iterate, bit for bit, as the z-wavefront order of a fused sweep
    (step t: colour 0 on plane t, colour 1 on plane t - 1, colour 2 on
    plane t - 2, colour 3 on plane t - 3): every vertex update reads the
    same values in both orders."""
    n = 6
    lv = mg.Level(3, n, [{'kind': 'sphere', 'center': (0.5, 0.45, 0.55), 'radius': 0.3, 'phase': 1}],
                  [1.0, 100.0], form)
    ijk = mesh.vertex_ijk(3, n)
    col = lv.colour
    rng = np.random.default_rng(5)
    x0 = rng.uniform(-1, 1, 3 * lv.N) * lv.free[:3 * lv.N]
    b = rng.uniform(-1, 1, 3 * lv.N) * lv.free[:3 * lv.N]
    phases = [np.flatnonzero(col == c) for c in range(4)]
    wave = [np.flatnonzero((col == c) & (ijk[:, 2] == t - c)) for t in range(n + 4) for c in range(4)]
    xa = _point_gs(lv, x0.copy(), b, phases)
    xb = _point_gs(lv, x0.copy(), b, wave)
    assert np.array_equal(xa, xb)
    assert not np.array_equal(xa, x0)


def test_smoother_equals_triangular_solves():
    """One Uzawa step (eq. Uzawa_smooth) equals: a forward then a backward
    triangular solve of the velocity block in (colour, component) order and
    a forward triangular solve of C in colour order (library routine
    spsolve_triangular), with p += omega delta."""
    lv = mg.Level(3, 4, SPHERE, [1.0, 100.0], 'strain')
    dim, N = 3, lv.N
    rng = np.random.default_rng(3)
    x = rng.uniform(-1, 1, 4 * N) * lv.free
    b = rng.uniform(-1, 1, 4 * N) * lv.free
    got = mg.smooth(lv, x, b, 1)
    # velocity: free dofs ordered by (colour, component, vertex)
    vid = np.arange(N)
    dofs = [k * N + vid[(lv.colour == c) & ~lv.disc.boundary]
            for c in range(4) for k in range(3)]
    order = np.concatenate(dofs)
    A = lv.A[order][:, order].tocsr()
    u, p = x[:3 * N].copy(), x[3 * N:].copy()
    rhs = (b[:3 * N] - lv.BT @ p)[order]
    uo = u[order]
    L = sp.tril(A, format='csr')
    U = sp.triu(A, format='csr')
    uo = uo + spla.spsolve_triangular(L, rhs - A @ uo, lower=True)
    uo = uo + spla.spsolve_triangular(U, rhs - A @ uo, lower=False)
    u[order] = uo
    porder = np.concatenate([vid[lv.colour == c] for c in range(4)])
    Cp = lv.C[porder][:, porder].tocsr()
    s = (lv.B @ u - lv.C @ p - b[3 * N:])[porder]
    delta = np.zeros(N)
    delta[porder] = spla.spsolve_triangular(sp.tril(Cp, format='csr'), s, lower=True)
    ref = np.concatenate([u, p + mg.OMEGA * delta])
    assert np.allclose(got, ref, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("dim", [2, 3])
def test_prolongation_is_p1_interpolation(dim):
    """Standard transfers (Sec. 5): P reproduces linear functions exactly,
    and for constant viscosity the Galerkin product P^T A_f P equals the
    rediscretised coarse Laplacian (nested P1 spaces)."""
    nc = 4
    P = mg.prolongation(dim, nc)
    g = np.arange(1, dim + 1) * 0.3
    lin_c = mesh.vertex_coords(dim, nc) @ g + 0.5
    lin_f = mesh.vertex_coords(dim, 2 * nc) @ g + 0.5
    assert np.allclose(P @ lin_c, lin_f, rtol=0, atol=1e-14)
    Af = assemble.Discretisation(dim, 2 * nc, [], [3.0]).mass()
    Ac = assemble.Discretisation(dim, nc, [], [3.0]).mass()
    assert abs(P.T @ Af @ P - Ac).max() < 1e-14
    Lf = assemble.Discretisation(dim, 2 * nc, [], [3.0]).stabilisation() / (2 * nc) ** -2
    Lc = assemble.Discretisation(dim, nc, [], [3.0]).stabilisation() / nc ** -2
    assert abs(P.T @ Lf @ P - Lc).max() < 1e-12 * abs(Lc).max()


def test_one_level_cycle_is_direct_solve():
    H = mg.Hierarchy(2, 1, 3, 3, SPLIT, [1.0, 10.0], 'interface')
    lv = H.levels[3]
    b = iss_inputs.random_rhs(2, 8, seed=2)
    x = H.vcycle(3, np.zeros_like(b), b)
    assert np.linalg.norm(lv.K @ x - b) < 1e-11 * np.linalg.norm(b)
    assert abs(np.dot(lv.weights, x[2 * lv.N:])) < 1e-12


def test_manufactured_solution_is_valid():
    """The 2D manufactured solution satisfies the interface problem of
    eq. stokes-strong-interface symbolically."""
    x, y, psi, p, curl, f = manufactured.symbols()
    for mu in (sy.Integer(10), sy.Integer(1)):
        u = (curl[0] / mu, curl[1] / mu)
        assert sy.simplify(sy.diff(u[0], x) + sy.diff(u[1], y)) == 0
        for a in range(2):
            r = -mu * (sy.diff(u[a], x, 2) + sy.diff(u[a], y, 2)) + sy.diff(p, (x, y)[a]) - f[a]
            assert sy.simplify(r) == 0
    half = sy.Rational(1, 2)
    for comp in curl:
        assert sy.simplify(comp.subs(x, half)) == 0
        for s in (0, 1):
            assert sy.simplify(comp.subs(x, s)) == 0 and sy.simplify(comp.subs(y, s)) == 0


def _manufactured_errors(form, n):
    D = assemble.Discretisation(2, n, SPLIT, [1.0, 10.0])
    X = mesh.vertex_coords(2, n)
    b = problem.rhs_from_nodal_force(2, n, D.elems, manufactured.force(X))
    K = D.stokes(form)
    lv = mg.Level(2, n, SPLIT, [1.0, 10.0], form)
    xh = mg.direct_solve(lv, b * D.free_mask())
    u_ex = manufactured.velocity(X, 10.0, 1.0).T.ravel()
    M = D.mass()
    e = (xh[:2 * D.N] - u_ex).reshape(2, D.N)
    err = np.sqrt(sum(ek @ (M @ ek) for ek in e))
    return err, xh, D


def test_manufactured_velocity_converges_at_second_order():
    """O(h^2) L2 velocity convergence of the consistent forms on the
    interface problem (compare the P1-P1 rates 1.79-1.97 of the paper's
    column tables)."""
    for form in ('interface', 'strain'):
        errs = [_manufactured_errors(form, n)[0] for n in (8, 16, 32, 64)]
        rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
        assert rates[-1] >= 1.8 and rates[-2] >= 1.8, (form, errs, rates)


def _solve_with_force(form, n, fn):
    D = assemble.Discretisation(2, n, SPLIT, [1.0, 10.0])
    X = mesh.vertex_coords(2, n)
    b = problem.rhs_from_nodal_force(2, n, D.elems, fn(X)) * D.free_mask()
    lv = mg.Level(2, n, SPLIT, [1.0, 10.0], form)
    return mg.direct_solve(lv, b), D


def test_gradient_form_is_inconsistent():
    """Sec. 1 / Sec. 4 tables: with a forcing like the paper's layer and
    column examples the gradient form converges to a different solution
    (relative difference does not vanish) while the interface form
    approaches the strain form at second order.  (The manufactured
    solution above is not used: mu grad u is continuous for it, so it
    happens to satisfy the gradient form's interface condition too.)"""
    fn = lambda X: np.stack([0 * X[:, 0], -np.cos(2 * np.pi * X[:, 0]) * np.sin(np.pi * X[:, 1])], 1)
    d_lap, d_tr = [], []
    for n in (16, 32, 64):
        xs, D = _solve_with_force('strain', n, fn)
        xl, _ = _solve_with_force('gradient', n, fn)
        xt, _ = _solve_with_force('interface', n, fn)
        M = D.mass()
        nrm = lambda v: np.sqrt(sum(vk @ (M @ vk) for vk in v.reshape(2, D.N)))
        d_lap.append(nrm(xl[:2 * D.N] - xs[:2 * D.N]) / nrm(xs[:2 * D.N]))
        d_tr.append(nrm(xt[:2 * D.N] - xs[:2 * D.N]) / nrm(xs[:2 * D.N]))
    assert d_lap[-1] > 0.7 * d_lap[0] and d_lap[-1] > 1e-2, d_lap
    # observed rates 1.6 and 1.5 (the paper's P1-P1 column table shows
    # 1.79-1.97 in 3D); the pin asks for clearly super-linear decay
    assert np.log2(d_tr[0] / d_tr[1]) > 1.3 and np.log2(d_tr[1] / d_tr[2]) > 1.3, d_tr


def test_buoyancy_load_total():
    """sum_j b_{j,z} = -rho * total volume of the buoyant elements; it tends
    to -4/3 pi r^3 under refinement."""
    n = 16
    D = assemble.Discretisation(3, n, SPHERE, [1.0, 10.0])
    b = problem.rhs_buoyancy(3, n, D.elems, D.phase_e, [1])
    assert np.isclose(b[2 * D.N:3 * D.N].sum(), -D.vol[D.phase_e == 1].sum(), rtol=1e-13)
    assert np.isclose(-b.sum(), 4.0 / 3.0 * np.pi * 0.3 ** 3, rtol=0.1)


def test_multigrid_rate_in_paper_regime():
    """Sec. 5 (contrast 10): the Uzawa V(3,3) cycle contracts with a rate
    near the paper's 0.24 for both consistent forms."""
    for form in ('interface', 'strain'):
        H = mg.Hierarchy(3, 1, 4, 3, SPHERE, [1.0, 10.0], form)
        rho = H.asymptotic_rate(25)
        assert rho < 0.35, (form, rho)


def test_fgmres_high_contrast_matches_direct():
    inc = iss_inputs.workload('sphere_3d', levels=4)
    H = mg.Hierarchy(3, 1, 4, 3, inc['inclusions'], inc['mu'], 'interface')
    lv = H.levels[4]
    b = iss_inputs.random_rhs(3, 16, seed=0)
    x, hist = mg.solve_fgmres(H, b)
    assert hist[-1] <= 1e-8 and len(hist) < 45
    xd = mg.direct_solve(lv, b)
    xn = problem.normalise_pressure(x, 3, 16, lv.weights)
    assert np.linalg.norm(xn - xd) < 1e-5 * np.linalg.norm(xd)


@pytest.mark.parametrize("dim", [2, 3])
def test_averaged_coarse_viscosity_is_galerkin(dim):
    """Coarse elements with the volume-averaged viscosity give exactly the
    Galerkin products of the fine operators (nested P1 spaces): P^T A_f P
    for every viscous form, and 4 P^T C_f P for the stabilisation (h^2
    doubles twice), with 1/mu averaged for C."""
    import scipy.sparse as sp
    inc = [{'kind': 'halfspace', 'axis': 0, 'threshold': 0.3, 'phase': 1}] if dim == 2 else SPHERE
    nc = 4
    Df = assemble.Discretisation(dim, 2 * nc, inc, [1.0, 300.0])
    mu_a, imu_a, _, _ = mg.averaged_coarse_viscosity(dim, nc, Df.mu_e, Df.imu_e, [1.0, 300.0])
    Dc = assemble.Discretisation(dim, nc, inc, [1.0, 300.0], mu_e=mu_a, imu_e=imu_a)
    P1 = mg.prolongation(dim, nc)
    Pv = sp.block_diag([P1] * dim).tocsr()
    for form in ("gradient", "strain", "tr"):
        G = Pv.T @ Df.viscous(form) @ Pv
        A = Dc.viscous(form)
        assert abs(G - A).max() <= 1e-12 * abs(A).max(), form
    Gc = 4.0 * (P1.T @ Df.stabilisation() @ P1)
    C = Dc.stabilisation()
    assert abs(Gc - C).max() <= 1e-12 * abs(C).max()
    # the element averages are genuinely mixed near the interface
    assert ((mu_a > 1.0) & (mu_a < 300.0)).any()


def test_binned_coarse_viscosity_bounds():
    """The table model of averaged_coarse_viscosity: without a table the
    representation is the averages themselves; with a table too small for
    the distinct mixed averages, pure viscosities stay exact and mixed ones
    move by less than the bin width (log spacing, 250 bins); with a table
    that holds them all, nothing moves."""
    Df = assemble.Discretisation(3, 16, SPHERE, [1.0, 1e4])
    mu_a, imu_a, mu_e, imu_e = mg.averaged_coarse_viscosity(3, 8, Df.mu_e, Df.imu_e, [1.0, 1e4])
    assert np.array_equal(mu_e, mu_a) and np.array_equal(imu_e, imu_a)
    pure = (mu_a == 1.0) | (mu_a == 1e4)
    nmixed = len(set(zip(mu_a[~pure], imu_a[~pure])))
    assert nmixed > 4
    _, _, mu_q, imu_q = mg.averaged_coarse_viscosity(3, 8, Df.mu_e, Df.imu_e, [1.0, 1e4], table=4)
    assert np.array_equal(mu_q[pure], mu_a[pure])
    width = np.log(mu_a[~pure].max() / mu_a[~pure].min()) / 250
    assert np.max(np.abs(np.log(mu_q[~pure] / mu_a[~pure]))) <= width + 1e-12
    _, _, mu_t, imu_t = mg.averaged_coarse_viscosity(3, 8, Df.mu_e, Df.imu_e, [1.0, 1e4], table=2 + nmixed)
    assert np.array_equal(mu_t[~pure], mu_a[~pure]) and np.array_equal(imu_t[~pure], imu_a[~pure])
    # pure elements take the problem's viscosity exactly (the average of
    # equal 1/mu values may be off by an ulp)
    assert np.allclose(imu_t[pure] * mu_t[pure], 1.0, rtol=1e-15, atol=0)


def test_binned_coarse_viscosity_changes_vcycle_boundedly():
    """Effect of the 254-entry viscosity table on the V-cycle: on the 64^3
    sinker (contrast 1e4, averaged coarse viscosity) the two levels below
    the 16^3 one hold more distinct averages than the table, so they are
    binned (relative width below 4%).  One V-cycle with the binned coarse
    levels differs from the one with exact averages by less than 5% of the
    correction it computes, and both contract the residual of the same
    right-hand side alike (ratio within 10%)."""
    import copy
    w = iss_inputs.workload('sinker_3d', levels=5)
    kw = dict(nu1=2, nu2=2, omega=0.6, coarse_mu='average', coarse_form='strain')
    args = (w['dim'], w['macro'], w['levels'], w['coarse'], w['inclusions'], w['mu'], 'interface')
    He = mg.Hierarchy(*args, **kw)
    # the same hierarchy with the table model on the coarse levels (the
    # finest level and the transfers are shared)
    Hb = copy.copy(He)
    Hb.levels = dict(He.levels)
    mu_f, imu_f = He.levels[w['levels']].disc.mu_e, He.levels[w['levels']].disc.imu_e
    for l in range(w['levels'] - 1, w['coarse'] - 1, -1):
        n = w['macro'] * 2 ** l
        mu_f, imu_f, mq, iq = mg.averaged_coarse_viscosity(3, n, mu_f, imu_f, w['mu'], table=254)
        Hb.levels[l] = mg.Level(3, n, w['inclusions'], w['mu'], He.levels[l].form, mu_e=mq, imu_e=iq)
    Hb.coarse_solver = mg.CoarseSolver(Hb.levels[w['coarse']])
    binned = [l for l in range(w['coarse'], w['levels'])
              if not np.array_equal(Hb.levels[l].disc.mu_e, He.levels[l].disc.mu_e)]
    assert binned, "the table should force binning on some coarse level"
    b = iss_inputs.random_rhs(3, w['n'], seed=5)
    x0 = np.zeros_like(b)
    xe = He.vcycle(w['levels'], x0, b)
    xb = Hb.vcycle(w['levels'], x0, b)
    assert np.linalg.norm(xb - xe) <= 0.05 * np.linalg.norm(xe)
    lv = He.levels[w['levels']]
    re = np.linalg.norm(mg.residual(lv, xe, b))
    rb = np.linalg.norm(mg.residual(lv, xb, b))
    assert abs(rb / re - 1.0) < 0.1, (re, rb)


@pytest.mark.parametrize("dim,n", [(2, 8), (3, 4)])
def test_incident_elements_by_brute_force(dim, n):
    """incident_elements (the candidate-cell search behind the sampled rows)
    returns exactly the lattice elements that contain a sample vertex:
    compared with a scan of every element; an interior vertex lies in d!
    2^d / ... = 6 (2D) or 24 (3D) elements (Kuhn lattice incidence)."""
    E = mesh.kuhn_elements(dim, n)
    N = mesh.num_vertices(dim, n)
    verts = np.unique(np.concatenate([[0, N - 1, N // 2], iss_inputs.sample_vertices(dim, n, 12, seed=3)]))
    got = mesh.incident_elements(dim, n, verts)
    ref = E[np.isin(E, verts).any(axis=1)]
    key = lambda A: sorted(map(tuple, np.sort(A, axis=1)))
    assert key(got) == key(ref)
    for v in verts:
        cnt = int((got == v).any(axis=1).sum())
        assert cnt == int((E == v).any(axis=1).sum())
        if not mesh.boundary_mask(dim, n)[v]:
            assert cnt == (6 if dim == 2 else 24)


@pytest.mark.parametrize("form", ["gradient", "strain", "interface"])
@pytest.mark.parametrize("dim,n", [(2, 16), (3, 8)])
def test_sampled_rows_equal_full_assembly(dim, n, form):
    """sampled_stokes_rows (the oracle of the full-size sampled parity tests)
    equals the rows of the globally assembled, Dirichlet-masked K x at
    boundary, interface and bulk vertices, for every form."""
    inc = SPLIT if dim == 2 else iss_inputs.workload('sinker_3d', levels=2)['inclusions']
    mu = [1.0, 300.0]
    D = assemble.Discretisation(dim, n, inc, mu)
    x = iss_inputs.random_vector(dim, n, seed=7)
    y = D.stokes(form) @ x
    bnd = np.nonzero(D.boundary)[0]
    itf = np.nonzero(D.interface & ~D.boundary)[0]
    blk = np.nonzero(~D.interface & ~D.boundary)[0]
    assert len(itf) > 0
    verts = np.unique(np.concatenate([bnd[::7], itf[::3], blk[::11]]))
    vs, Y = assemble.sampled_stokes_rows(dim, n, inc, mu, verts, form, x)
    N = D.N
    ref = np.stack([y[f * N + vs] for f in range(dim + 1)])
    scale = np.abs(ref).max()
    assert np.abs(Y - ref).max() <= 1e-13 * scale


def test_interface_form_inertia():
    """Characterisation behind the high-contrast solver choices: the strain
    system has the saddle-point inertia (N_p - 1 negative eigenvalues); the
    interface (a_tr) system keeps it at contrast 10 but gains extra negative
    eigenvalues at contrast 1e3 on an unresolved 8-sphere geometry (a_tr is
    not positive semi-definite, Sec. 3)."""
    w = iss_inputs.workload('sinker_3d', levels=2)
    counts = {}
    for mu_in in (10.0, 1e3):
        for form in ('strain', 'interface'):
            D = assemble.Discretisation(3, w['n'], w['inclusions'], [1.0, mu_in])
            K = D.stokes(form)
            f = D.free_mask()
            Kf = K[f][:, f].toarray()
            s = 1.0 / np.sqrt(np.abs(np.diag(Kf)))
            ev = np.linalg.eigvalsh(s[:, None] * Kf * s[None, :])
            counts[(mu_in, form)] = int((ev < -1e-12).sum())
    npres = D.N
    assert counts[(10.0, 'strain')] == npres - 1
    assert counts[(1e3, 'strain')] == npres - 1
    assert counts[(10.0, 'interface')] == npres - 1
    assert counts[(1e3, 'interface')] > npres - 1


def test_coarse_rhs_modification_brings_strain_towards_tr():
    """Sec. 5, coarse grid solver: with the strain form on the coarse grid,
    the momentum right-hand side r_1 + B^T M^-1 r_2 (M the lumped
    (1/mu)-weighted pressure mass; the paper's minus sign belongs to its
    opposite sign of B) makes the strain-form solution closer to the a_tr
    solution of the same right-hand side than the unmodified one, and the
    opposite sign moves it away.  9^3 sinker, contrasts 10 and 1e3."""
    w = iss_inputs.workload('sinker_3d', levels=2)
    for mu_in in (10.0, 1e3):
        mu = [1.0, mu_in]
        lt = mg.Level(3, w['n'], w['inclusions'], mu, 'interface')
        ls = mg.Level(3, w['n'], w['inclusions'], mu, 'strain')
        N = lt.N
        r = np.random.default_rng(1).uniform(-1, 1, 4 * N) * lt.free
        xt = mg.direct_solve(lt, r)
        d = {}
        for sgn in (0, 1, -1):
            rm = r.copy()
            rm[:3 * N] += sgn * (ls.BT @ (r[3 * N:] / lt.weights))
            xs = mg.direct_solve(ls, rm)
            d[sgn] = np.linalg.norm(xs[:3 * N] - xt[:3 * N]) / np.linalg.norm(xt[:3 * N])
        assert d[1] < 0.85 * d[0] and d[-1] > d[0], (mu_in, d)
