"""Explicit global assembly of the discrete Stokes operators (COO -> CSR).

Global numbering: velocity dof (vertex v, component k) -> k * N + v, pressure
dof v -> d * N + v, N = number of lattice vertices.  This is the field-major
layout [u_1 | .. | u_d | p] used by every vector of the project.

The saddle-point system of Sec. 5 is K = [[A, B^T], [B, -C]] with A from one
of the viscous forms, B the weak divergence (eq. weaks) and C the pressure
stabilisation.  Fixed velocity dofs (eq. boundary: every component on the
boundary for no-slip, the normal component for free-slip; see
mesh.fixed_velocity) are handled by masking: rows and columns of fixed dofs
are zero, so K acts on vectors whose fixed entries are ignored and returns
zero there.
"""
import numpy as np
import scipy.sparse as sp

from . import fem, mesh, problem

FORMS = ('gradient', 'strain', 'interface', 'tr')


class Discretisation:
    """Kuhn lattice of n cells per axis on the unit cube/square with the
    element viscosities of a list of inclusions (see problem.element_phase).

    ``elems`` may be a subset of the lattice elements (row sampling): then
    only rows of vertices whose incident elements are all present are
    meaningful."""

    def __init__(self, dim, n, inclusions, mu_table, elems=None, mu_e=None, imu_e=None, bc='noslip'):
        self.dim, self.n = dim, n
        self.bc = bc
        self.N = mesh.num_vertices(dim, n)
        self.h = 1.0 / n
        self.elems = mesh.kuhn_elements(dim, n) if elems is None else elems
        self.inclusions = inclusions
        self.mu_table = np.asarray(mu_table, dtype=np.float64)
        self.phase_e = problem.element_phase(dim, n, self.elems, inclusions)
        # per-element viscosity (viscous blocks) and inverse viscosity
        # (stabilisation, pressure weights); by default from the phases
        self.mu_e = self.mu_table[self.phase_e] if mu_e is None else np.asarray(mu_e, np.float64)
        self.imu_e = 1.0 / self.mu_e if imu_e is None else np.asarray(imu_e, np.float64)
        X = mesh.vertex_coords(dim, n)[self.elems]
        self.G, self.vol = fem.simplex_geometry(X)
        self.interface = problem.interface_vertices(dim, n, self.elems, self.mu_e)
        self.boundary = mesh.boundary_mask(dim, n)
        self.fixed = mesh.fixed_velocity(dim, n, bc)     # (dim, N)

    # -- dof bookkeeping ---------------------------------------------------
    @property
    def ndof(self):
        return (self.dim + 1) * self.N

    def free_mask(self):
        """Velocity dofs that are not fixed, and every pressure dof."""
        f = np.ones(self.ndof, dtype=bool)
        f[:self.dim * self.N] = ~self.fixed.ravel()
        return f

    def _velocity_dofs(self):
        d = self.dim
        return (np.arange(d)[None, None, :] * self.N
                + self.elems[:, :, None]).reshape(len(self.elems), (d + 1) * d)

    # -- blocks ------------------------------------------------------------
    def _coo(self, Ke, rdof, cdof, shape, chunk=200000):
        out = None
        for s in range(0, len(Ke), chunk):
            K = Ke[s:s + chunk]
            r = np.broadcast_to(rdof[s:s + chunk, :, None], K.shape)
            c = np.broadcast_to(cdof[s:s + chunk, None, :], K.shape)
            M = sp.coo_matrix((K.ravel(), (r.ravel(), c.ravel())), shape=shape).tocsr()
            out = M if out is None else out + M
        if out is None:
            out = sp.csr_matrix(shape)
        out.sum_duplicates()
        return out

    def viscous(self, form):
        """Velocity block A (dN x dN), unmasked.

        'gradient'  : (mu grad u, grad v) on every row (inconsistent, Sec. 1)
        'strain'    : a_sym, eq. standard
        'tr'        : a_tr, eq. newbil
        'interface' : the row-wise operator of eq. equivalence-stencil --
                      rows of interface and boundary vertices from a_tr,
                      every other row from the isoviscous Laplacian
                      (mu grad u, grad v).  The full rows on the boundary are
                      those Sec. 2.2 asks for on Gamma_F; on Dirichlet
                      vertices the rows are masked anyway.
        """
        d, N = self.dim, self.N
        vd = self._velocity_dofs()
        if form in ('gradient', 'strain', 'tr'):
            key = {'gradient': 'lap', 'strain': 'sym', 'tr': 'tr'}[form]
            Ke = fem.viscous_element_matrices(self.G, self.vol, self.mu_e, key)
            return self._coo(Ke, vd, vd, (d * N, d * N))
        if form == 'interface':
            A_lap = self.viscous('gradient')
            A_tr = self.viscous('tr')
            rows_if = np.tile(self.interface | self.boundary, d).astype(np.float64)
            return sp.diags(rows_if) @ A_tr + sp.diags(1.0 - rows_if) @ A_lap
        raise ValueError(form)

    def divergence(self):
        """B (N x dN): (B u)_j = -(div u, lambda_j)."""
        d, N = self.dim, self.N
        Be = fem.divergence_element_matrices(self.G, self.vol)
        return self._coo(Be, self.elems, self._velocity_dofs(), (N, d * N))

    def stabilisation(self):
        """C (N x N): c(p, q) = sum_T beta h^2/mu_T (grad p, grad q)_T."""
        Ce = fem.stabilisation_element_matrices(self.G, self.vol, 1.0 / self.imu_e, self.h)
        return self._coo(Ce, self.elems, self.elems, (self.N, self.N))

    def mass(self):
        Me = fem.mass_element_matrices(self.vol, self.dim)
        return self._coo(Me, self.elems, self.elems, (self.N, self.N))

    def stokes(self, form, masked=True):
        """K = [[A, B^T], [B, -C]]; with masked=True rows and columns of
        Dirichlet velocity dofs are zeroed."""
        A = self.viscous(form)
        B = self.divergence()
        C = self.stabilisation()
        K = sp.bmat([[A, B.T], [B, -C]], format='csr')
        if masked:
            D = sp.diags(self.free_mask().astype(np.float64))
            K = (D @ K @ D).tocsr()
        K.eliminate_zeros()
        return K

    def velocity_operator(self, form, masked=True):
        A = self.viscous(form)
        if masked:
            D = sp.diags((~self.fixed.ravel()).astype(np.float64))
            A = (D @ A @ D).tocsr()
        A.eliminate_zeros()
        return A


def sampled_rows(dim, n, inclusions, mu_table, verts, bc='noslip'):
    """A Discretisation restricted to the elements incident to ``verts``.

    Rows of ``verts`` of any operator assembled from it equal the rows of
    the full assembly (a row only receives contributions from elements that
    contain its vertex); all other rows are incomplete and must not be used.
    """
    elems = mesh.incident_elements(dim, n, verts)
    return Discretisation(dim, n, inclusions, mu_table, elems=elems, bc=bc)


def sampled_stokes_rows(dim, n, inclusions, mu_table, verts, form, x, bc='noslip'):
    """Rows of y = K x at the vertices ``verts`` (all d+1 fields) without
    assembling K globally: the element matrices of the elements incident to
    the sample are scattered only into sample rows.  Dirichlet masking as in
    Discretisation.stokes.  Returns Y with Y[f, i] = y[f * N + verts[i]]."""
    verts = np.unique(np.asarray(verts, dtype=np.int64))
    D = sampled_rows(dim, n, inclusions, mu_table, verts, bc=bc)
    N = D.N
    d = dim
    lookup = {int(v): i for i, v in enumerate(verts)}
    key = {'gradient': 'lap', 'strain': 'sym', 'interface': 'tr', 'tr': 'tr'}[form]
    Ke = fem.viscous_element_matrices(D.G, D.vol, D.mu_e, key)
    if form == 'interface':
        # rows of non-interface vertices come from the Laplacian form
        Kl = fem.viscous_element_matrices(D.G, D.vol, D.mu_e, 'lap')
    Be = fem.divergence_element_matrices(D.G, D.vol)
    Ce = fem.stabilisation_element_matrices(D.G, D.vol, D.mu_e, D.h)
    fixed = D.fixed
    Y = np.zeros((d + 1, len(verts)))
    E = D.elems
    for e in range(len(E)):
        ev = E[e]
        for a in range(d + 1):
            va = int(ev[a])
            if va not in lookup:
                continue
            i = lookup[va]
            # velocity rows (zero for fixed components)
            src = Ke if (form != 'interface' or D.interface[va] or D.boundary[va]) else Kl
            for l in range(d):
                if fixed[l, va]:
                    continue
                acc = 0.0
                for b in range(d + 1):
                    vb = int(ev[b])
                    for k in range(d):
                        if not fixed[k, vb]:
                            acc += src[e, a * d + l, b * d + k] * x[k * N + vb]
                    acc += Be[e, b, a * d + l] * x[d * N + vb]
                Y[l, i] += acc
            # pressure row
            acc = 0.0
            for b in range(d + 1):
                vb = int(ev[b])
                for k in range(d):
                    if not fixed[k, vb]:
                        acc += Be[e, a, b * d + k] * x[k * N + vb]
                acc -= Ce[e, a, b] * x[d * N + vb]
            Y[d, i] += acc
    return verts, Y
