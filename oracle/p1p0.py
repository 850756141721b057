"""Stabilised P1-P0 discretisation (Sec. 3): P1 velocity, piecewise constant
pressure, the interior-penalty stabilisation of eq. stabc and the local
flux post-process that restores element-wise mass conservation (oracle;
test infrastructure only).

Pressure unknowns live on the elements of the Kuhn lattice, in the order of
mesh.kuhn_elements (cell x fastest, then the axis-order permutations).  The
system is K = [[A, B0^T], [B0, -C]] with
  * A one of the viscous forms of assemble.Discretisation (the discrete form
    of Sec. 3 takes a_tr; the others serve as references),
  * (B0 u)_T = b(u, 1_T) = -(div u, 1)_T = -|T| sum_a grad(lambda_a) . u_a,
  * c(p, q) = gamma sum_i 1/(2 mu_i) sum_{F interior to Omega_i}
    |T1||T2| / (|T1| + |T2|) [p]_F [q]_F (eq. stabc): only facets between
    two elements of equal viscosity are penalised, so no pressure jump across
    the interface is penalised.

The post-processed flux through facet F of element T is
  int_F j_{F;T} = int_F u_h . n_T + gamma / (2 mu) |T||T^F| / (|T| + |T^F|)
                  (p_T - p_{T^F})
(the second term only on penalised facets); their sum over the facets of T
is -(B0 u - C p)_T, zero for a solution of the system with g = 0.
"""
import numpy as np
import scipy.sparse as sp

from . import assemble, fem, mesh


def face_neighbours(dim, n, elems=None):
    """(E, d+1) array: the element across the facet opposite local vertex a
    of each element, -1 on the boundary.  Found by matching the sorted
    vertex sets of the facets."""
    E = mesh.kuhn_elements(dim, n) if elems is None else elems
    ne = len(E)
    keys, owner, loc = [], [], []
    for a in range(dim + 1):
        f = np.sort(np.delete(E, a, axis=1), axis=1)
        keys.append(f)
        owner.append(np.arange(ne))
        loc.append(np.full(ne, a))
    keys = np.concatenate(keys)
    owner = np.concatenate(owner)
    loc = np.concatenate(loc)
    _, inv = np.unique(keys, axis=0, return_inverse=True)
    inv = inv.ravel()
    order = np.argsort(inv, kind='stable')
    si = inv[order]
    # a facet shared by two elements appears twice, consecutively after sorting
    pair = np.nonzero(si[:-1] == si[1:])[0]
    i, j = order[pair], order[pair + 1]
    nb = -np.ones((ne, dim + 1), dtype=np.int64)
    nb[owner[i], loc[i]] = owner[j]
    nb[owner[j], loc[j]] = owner[i]
    return nb


class P1P0:
    def __init__(self, dim, n, inclusions, mu_table, gamma=1.0, bc='noslip', mu_e=None):
        self.d = assemble.Discretisation(dim, n, inclusions, mu_table, mu_e=mu_e, bc=bc)
        self.dim, self.n, self.N = dim, n, self.d.N
        self.gamma = gamma
        self.E = self.d.elems
        self.ne = len(self.E)
        self.nb = face_neighbours(dim, n, self.E)
        self.vol = self.d.vol
        self.mu_e = self.d.mu_e

    @property
    def ndof(self):
        return self.dim * self.N + self.ne

    def free_mask(self):
        f = np.ones(self.ndof, dtype=bool)
        f[:self.dim * self.N] = ~self.d.fixed.ravel()
        return f

    def divergence(self):
        """B0 (E x dN): (B0 u)_T = -|T| sum_a grad(lambda_a) . u_a."""
        d, N = self.dim, self.N
        G = self.d.G                                        # (E, d+1, d)
        rows = np.repeat(np.arange(self.ne), (d + 1) * d)
        cols = (np.arange(d)[None, None, :] * N + self.E[:, :, None]).ravel()
        vals = (-self.vol[:, None, None] * G).ravel()
        return sp.csr_matrix((vals, (rows, cols)), shape=(self.ne, d * N))

    def penalty_weights(self):
        """(E, d+1): the weight of the term (p_T - p_T') of each facet, zero
        on boundary facets and on facets between different viscosities."""
        w = np.zeros((self.ne, self.dim + 1))
        for a in range(self.dim + 1):
            j = self.nb[:, a]
            ok = j >= 0
            jj = np.where(ok, j, 0)
            same = ok & (self.mu_e[jj] == self.mu_e)
            v1, v2 = self.vol, self.vol[jj]
            w[:, a] = np.where(same, self.gamma / (2.0 * self.mu_e) * v1 * v2 / (v1 + v2), 0.0)
        return w

    def stabilisation(self):
        """C (E x E) of eq. stabc."""
        w = self.penalty_weights()
        rows, cols, vals = [], [], []
        for a in range(self.dim + 1):
            j = self.nb[:, a]
            sel = w[:, a] != 0
            t = np.nonzero(sel)[0]
            rows += [t, t]
            cols += [t, j[sel]]
            vals += [w[sel, a], -w[sel, a]]
        return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                             shape=(self.ne, self.ne))

    def stokes(self, form, masked=True):
        A = self.d.viscous(form)
        B = self.divergence()
        C = self.stabilisation()
        K = sp.bmat([[A, B.T], [B, -C]], format='csr')
        if masked:
            D = sp.diags(self.free_mask().astype(np.float64))
            K = (D @ K @ D).tocsr()
        K.eliminate_zeros()
        return K

    def fluxes(self, x):
        """(E, d+1): int_F j_{F;T} for the facet opposite each local vertex."""
        d, N = self.dim, self.N
        u = x[:d * N].reshape(d, N)
        p = x[d * N:]
        G = self.d.G
        U = u[:, self.E].transpose(1, 2, 0)                 # (E, d+1, d)
        out = np.empty((self.ne, d + 1))
        for a in range(d + 1):
            # int_F u_h . n_T = -|T| grad(lambda_a) . sum_{b != a} u_b
            s = U.sum(axis=1) - U[:, a, :]
            out[:, a] = -self.vol * np.einsum('ed,ed->e', G[:, a, :], s)
        w = self.penalty_weights()
        for a in range(d + 1):
            j = self.nb[:, a]
            pj = p[np.where(j >= 0, j, 0)]
            out[:, a] += w[:, a] * (p - pj)
        return out

    def pressure_weights(self):
        """int 1_T / mu = |T| / mu_T: the constraint of the space Q (Sec. 1)."""
        return self.vol / self.mu_e


def direct_solve(P, form, b):
    """x = K^-1 b on the free dofs, the pressure fixed by sum_T |T| p_T / mu_T
    = 0 through a border row."""
    K = P.stokes(form)
    free = P.free_mask()
    idx = np.nonzero(free)[0]
    w = np.zeros(P.ndof)
    w[P.dim * P.N:] = P.pressure_weights()
    Kf = K[idx][:, idx]
    wf = w[idx]
    Kb = sp.bmat([[Kf, sp.csr_matrix(wf[:, None])], [sp.csr_matrix(wf[None, :]), None]], format='csc')
    import scipy.sparse.linalg as spla
    z = spla.spsolve(Kb, np.append(b[idx], 0.0))
    x = np.zeros(P.ndof)
    x[idx] = z[:-1]
    return x


# --- Couette flow with an interface (Sec. 4) -----------------------------------

def couette_exact(X, mu1, mu2):
    """u = (1/2 (1 - x^2), x y, 0), p = 2 x mu - (mu1 + mu2) / 2 on
    (0,1) x (-1/2,1/2) x (0,1), mu = mu1 for y < 0 and mu2 for y > 0."""
    x, y = X[..., 0], X[..., 1]
    mu = np.where(y < 0, mu1, mu2)
    u = np.stack([0.5 * (1 - x * x), x * y, np.zeros_like(x)], axis=-1)
    p = 2 * x * mu - 0.5 * (mu1 + mu2)
    return u, p, mu


def _tet_rule(order=4):
    """Collapsed (Duffy) Gauss rule on the unit tetrahedron: points (Q, 3)
    in barycentric-free reference coordinates and weights (Q,), exact for
    polynomials of degree <= 2 order - 3 (4 -> degree 5)."""
    g, wg = np.polynomial.legendre.leggauss(order)
    g, wg = 0.5 * (g + 1.0), 0.5 * wg
    pts, wts = [], []
    for i, a in enumerate(g):
        for j, b in enumerate(g):
            for k, c in enumerate(g):
                x = a
                y = b * (1 - a)
                z = c * (1 - a) * (1 - b)
                pts.append((x, y, z))
                wts.append(wg[i] * wg[j] * wg[k] * (1 - a) ** 2 * (1 - b))
    return np.array(pts), np.array(wts)


def couette_problem(level, mu1=1.0, mu2=1e-3, gamma=1.0, form='interface'):
    """The Couette benchmark of Sec. 4 on the Kuhn lattice with n = 4 2^level
    (h = 1/4 at level 0), the lattice shifted by -1/2 in y, Dirichlet data
    of the exact solution on the whole boundary (lifted into the right-hand
    side).  Returns the discretisation, the discrete solution and the errors
    (||u - u_h||_0, ||u - u_h||_V, ||p - p_h||_Q) by the collapsed Gauss
    rule (exact for these polynomial integrands)."""
    n = 4 * 2 ** level
    inc = [{'kind': 'halfspace', 'axis': 1, 'threshold': 0.5, 'phase': 1}]
    P = P1P0(3, n, inc, [mu2, mu1], gamma=gamma)
    N = P.N
    Xl = mesh.vertex_coords(3, n)
    Xp = Xl - np.array([0.0, 0.5, 0.0])
    ue, _, _ = couette_exact(Xp, mu1, mu2)
    fixed = P.d.fixed.ravel()
    xg = np.zeros(P.ndof)
    xg[:3 * N] = np.where(fixed, ue.T.ravel(), 0.0)
    # load of f = (3 mu, 0, 0): int_T f lambda_a = 3 mu_T |T| / 4
    b = np.zeros(P.ndof)
    np.add.at(b, P.E.ravel(), np.repeat(3.0 * P.mu_e * P.vol / 4.0, 4))
    K = P.stokes(form, masked=False)
    rhs = (b - K @ xg) * P.free_mask()
    x = direct_solve(P, form, rhs) + xg
    return P, x, couette_errors(P, x, mu1, mu2)


def couette_errors(P, x, mu1, mu2):
    N, E = P.N, P.E
    Xl = mesh.vertex_coords(3, P.n)
    shift = np.array([0.0, 0.5, 0.0])
    pts, wts = _tet_rule(4)
    Xe = Xl[E]                                                  # (E, 4, 3)
    J = Xe[:, 1:, :] - Xe[:, :1, :]                             # rows: edge vectors
    detJ = np.abs(np.linalg.det(J))
    lam = np.concatenate([1 - pts.sum(axis=1, keepdims=True), pts], axis=1)   # (Q, 4)
    Xq = np.einsum('qa,eak->eqk', lam, Xe) - shift              # physical points (E, Q, 3)
    u = x[:3 * N].reshape(3, N)
    uh = np.einsum('qa,kea->eqk', lam, u[:, E])                 # (E, Q, 3)
    ue, pe, mu = couette_exact(Xq, mu1, mu2)
    mu_T = P.mu_e[:, None]
    # velocity L2
    l2 = np.sum(detJ[:, None] * wts[None, :] * np.sum((ue - uh) ** 2, axis=2))
    # energy a_sym(e, e) = sum_T int 2 mu |eps(e)|^2; grad u_h per element
    G = P.d.G
    grad_h = np.einsum('eak,iea->eik', G, u[:, E])              # (E, i, k) = d u_i / d x_k
    x_, y_ = Xq[..., 0], Xq[..., 1]
    grad_e = np.zeros(Xq.shape[:2] + (3, 3))
    grad_e[..., 0, 0] = -x_
    grad_e[..., 1, 0] = y_
    grad_e[..., 1, 1] = x_
    D = grad_e - grad_h[:, None, :, :]
    eps = 0.5 * (D + np.swapaxes(D, -1, -2))
    en = np.sum(detJ[:, None] * wts[None, :] * 2.0 * mu_T * np.sum(eps ** 2, axis=(2, 3)))
    # pressure, after matching the weighted means int p / mu
    ph = x[3 * N:]
    wq = detJ[:, None] * wts[None, :] / mu_T
    c = (np.sum(wq * pe) - np.sum(wq * ph[:, None])) / np.sum(wq)
    pq = np.sum(detJ[:, None] * wts[None, :] * (pe - ph[:, None] - c) ** 2 / (2.0 * mu_T))
    return np.sqrt(l2), np.sqrt(en), np.sqrt(pq)
