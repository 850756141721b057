"""All-at-once Uzawa multigrid of Sec. 5 on explicitly assembled matrices.

Smoothing step (eq. Uzawa_smooth):
    u <- u + A_hat^{-1} (f - A u - B^T p)
    p <- p + S_hat^{-1} (B u - C p - g)
A_hat is one symmetric Gauss-Seidel sweep on the velocity block; S_hat is
one forward Gauss-Seidel sweep on the stabilisation block C started from
zero, damped by the factor omega = 0.3 (Sec. 5, eq. Uzawa_smooth).

Readings taken where Sec. 5 leaves the choice open:
  * ordering: the paper's symmetric, parallel red-black style row-wise
    Gauss-Seidel becomes a global multicolour Gauss-Seidel with colour
    (i + j [+ k]) mod (d + 1); the forward sweep visits colours 0..d and,
    inside a vertex, components 0..d-1; the backward sweep is the exact
    reverse (colours d..0, components d-1..0).  The hybrid variant (Jacobi
    between processes) is not used because it depends on the partition.
  * S_hat: delta solves (D_C + L_C) delta = B u - C p - g in the same colour
    order, then p += omega * delta.
  * transfers: prolongation is P1 interpolation between nested Kuhn
    lattices, restriction its transpose; fixed velocity entries are zeroed
    after restriction.
  * coarse operators: rediscretisation with the centroid rule on each level,
    or with the volume-averaged fine viscosity (Galerkin for nested P1).
  * forms per level: the finest level uses the form of the call; the levels
    in between use ``mid_form`` (default: the same form); the coarsest uses
    ``coarse_form`` (default: that of the levels above), which expresses the
    swap to the strain form on the coarse grid of Sec. 5.
  * coarse solve: direct, on the free dofs bordered by the pressure
    constraint sum_j w_j p_j = 0 (a direct coarse solver is the case the
    paper calls unproblematic, Sec. 5), or the preconditioned MINRES of
    Sec. 5 (krylov.py).
  * cycle: V(3,3) on every level ("V_var" is not defined further).
  * stopping: Euclidean norm of b - K x over all dofs <= rtol * ||b||.
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from . import assemble, mesh, problem

OMEGA = 0.3


def colours(dim, n):
    ijk = mesh.vertex_ijk(dim, n)
    return ijk.sum(axis=1) % (dim + 1)


def prolongation(dim, n_coarse):
    """P1 interpolation from the Kuhn lattice with n_coarse cells per axis
    to the one with 2 n_coarse cells: P[f, c] = lambda_c(x_f), the coarse
    hat function of vertex c evaluated at fine vertex f.  Built by locating
    each fine vertex in a coarse simplex and taking its barycentric
    coordinates (one scalar field; apply per field)."""
    nc, nf = n_coarse, 2 * n_coarse
    xf = mesh.vertex_coords(dim, nf)
    cell = np.minimum(np.floor(xf * nc).astype(np.int64), nc - 1)
    off = mesh.kuhn_offsets(dim)                               # (S, d+1, d)
    rows, cols, vals = [], [], []
    found = np.zeros(len(xf), dtype=bool)
    for s in range(off.shape[0]):
        vijk = cell[:, None, :] + off[s][None]                 # (Nf, d+1, d)
        X = vijk / nc
        M = np.concatenate([np.ones(X.shape[:2] + (1,)), X], axis=2)
        rhs = np.concatenate([np.ones((len(xf), 1)), xf], axis=1)[:, :, None]
        lam = np.linalg.solve(np.transpose(M, (0, 2, 1)), rhs)[:, :, 0]
        ok = np.all(lam > -1e-12, axis=1) & ~found
        found |= ok
        vid = mesh.vertex_index(dim, nc, vijk)
        for a in range(dim + 1):
            sel = ok & (np.abs(lam[:, a]) > 1e-12)
            rows.append(np.nonzero(sel)[0])
            cols.append(vid[sel, a])
            vals.append(lam[sel, a])
    assert found.all()
    Nf, Nc = mesh.num_vertices(dim, nf), mesh.num_vertices(dim, nc)
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(Nf, Nc))


def parent_elements(dim, n_coarse):
    """Index of the coarse Kuhn element (n_coarse cells per axis) that
    contains each element of the once-refined lattice.  The meshes are
    nested, so a fine centroid lies strictly inside its parent; the parent
    is found by barycentric coordinates in the simplices of its cell."""
    nf = 2 * n_coarse
    Ef = mesh.kuhn_elements(dim, nf)
    cen = mesh.vertex_coords(dim, nf)[Ef].mean(axis=1)
    cell = np.minimum(np.floor(cen * n_coarse).astype(np.int64), n_coarse - 1)
    off = mesh.kuhn_offsets(dim)
    parent = -np.ones(len(Ef), dtype=np.int64)
    cell_id = mesh.vertex_index(dim, n_coarse - 1, cell)
    for s in range(off.shape[0]):
        X = (cell[:, None, :] + off[s][None]) / n_coarse
        M = np.concatenate([np.ones(X.shape[:2] + (1,)), X], axis=2)
        rhs = np.concatenate([np.ones((len(cen), 1)), cen], axis=1)[:, :, None]
        lam = np.linalg.solve(np.transpose(M, (0, 2, 1)), rhs)[:, :, 0]
        ok = np.all(lam > 1e-12, axis=1) & (parent < 0)
        parent[ok] = cell_id[ok] * off.shape[0] + s
    assert (parent >= 0).all()
    return parent


def averaged_coarse_viscosity(dim, n_coarse, mu_f, imu_f, pure_values, table=None, nbins=250):
    """Coarse-element viscosity as the volume average over the nested fine
    elements (equal volumes under uniform refinement), and the same for
    1/mu.  For nested P1 spaces the viscous block assembled with these
    averages equals the Galerkin product P^T A P.

    Returns the averages (mu, 1/mu) and their representation on the level.
    With ``table=None`` (the definition) the representation is the averages
    themselves.  With a table size, it models a level that stores at most
    ``table`` distinct viscosities: averages equal to a viscosity of the
    problem (pure elements) are kept exactly, the distinct mixed averages
    are kept exactly if they fit the table, and otherwise they are grouped
    into ``nbins`` logarithmically spaced bins between the smallest and
    largest mixed average, every member of a bin taking the bin's mean of mu
    and of 1/mu.  This approximation is used only to bound its effect on the
    V-cycle (a test), never as the reference."""
    parent = parent_elements(dim, n_coarse)
    nce = n_coarse ** dim * (6 if dim == 3 else 2)
    kids = np.bincount(parent, minlength=nce)
    mu_avg = np.bincount(parent, mu_f, minlength=nce) / kids
    imu_avg = np.bincount(parent, imu_f, minlength=nce) / kids
    pure = np.zeros(nce, dtype=bool)
    mu_q, imu_q = mu_avg.copy(), imu_avg.copy()
    if table is None:
        return mu_avg, imu_avg, mu_q, imu_q
    npure = 0
    for v in sorted(set(pure_values)):
        hit = (np.abs(mu_avg - v) <= 1e-14 * v) & (np.abs(imu_avg * v - 1.0) < 1e-12)
        npure += bool(hit.any())
        pure |= hit
        mu_q[hit], imu_q[hit] = v, 1.0 / v
    nmixed = len(set(zip(mu_avg[~pure].tolist(), imu_avg[~pure].tolist())))
    if (~pure).any() and npure + nmixed > table:
        lm = np.log(mu_avg[~pure])
        lo, hi = lm.min(), lm.max()
        t = (lm - lo) / (hi - lo) if hi > lo else np.zeros_like(lm)
        b = np.minimum(nbins - 1, (t * nbins).astype(np.int64))
        cnt = np.bincount(b, minlength=nbins)
        bm = np.bincount(b, mu_avg[~pure], minlength=nbins) / np.maximum(cnt, 1)
        bi = np.bincount(b, imu_avg[~pure], minlength=nbins) / np.maximum(cnt, 1)
        mu_q[~pure], imu_q[~pure] = bm[b], bi[b]
    return mu_avg, imu_avg, mu_q, imu_q


class Level:
    def __init__(self, dim, n, inclusions, mu_table, form, mu_e=None, imu_e=None, bc='noslip'):
        self.disc = assemble.Discretisation(dim, n, inclusions, mu_table, mu_e=mu_e, imu_e=imu_e, bc=bc)
        d = self.disc
        self.dim, self.n, self.N = dim, n, d.N
        self.form = form
        self.A = d.velocity_operator(form)
        D = sp.diags((~d.fixed.ravel()).astype(np.float64))
        self.B = (d.divergence() @ D).tocsr()
        self.BT = self.B.T.tocsr()
        self.C = d.stabilisation()
        self.K = sp.bmat([[self.A, self.BT], [self.B, -self.C]], format='csr')
        self.Adiag = self.A.diagonal()
        self.Cdiag = self.C.diagonal()
        self.colour = colours(dim, n)
        self.free = d.free_mask()
        self.weights = problem.pressure_weights(dim, n, d.elems, 1.0 / d.imu_e)


def split(x, dim, N):
    return x[:dim * N], x[dim * N:]


def smooth(lv, x, b, nsteps=1, omega=OMEGA):
    """nsteps Uzawa smoothing steps in place order of the module docstring."""
    dim, N = lv.dim, lv.N
    x = np.array(x, dtype=np.float64, copy=True)
    for _ in range(nsteps):
        u, p = split(x, dim, N)
        f, g = split(b, dim, N)
        rhs = f - lv.BT @ p
        order = [(c, k) for c in range(dim + 1) for k in range(dim)]
        for c, k in order + order[::-1]:
            rows = k * N + np.nonzero((lv.colour == c) & lv.free[k * N:(k + 1) * N])[0]
            r = rhs[rows] - lv.A[rows] @ u
            u[rows] += r / lv.Adiag[rows]
        s = lv.B @ u - lv.C @ p - g
        delta = np.zeros(N)
        for c in range(dim + 1):
            rows = np.nonzero(lv.colour == c)[0]
            delta[rows] = (s[rows] - lv.C[rows] @ delta) / lv.Cdiag[rows]
        p += omega * delta
        x[:dim * N], x[dim * N:] = u, p
    return x


def residual(lv, x, b):
    return b - lv.K @ x


class CoarseSolver:
    """Dense LU of the free-dof coarse matrix bordered with the weighted
    pressure-mean row."""

    def __init__(self, lv):
        self.lv = lv
        self.idx = np.nonzero(lv.free)[0]
        Kf = lv.K[self.idx][:, self.idx].toarray()
        w = np.zeros(lv.K.shape[0])
        w[lv.dim * lv.N:] = lv.weights
        wf = w[self.idx]
        m = len(self.idx)
        Kb = np.zeros((m + 1, m + 1))
        Kb[:m, :m] = Kf
        Kb[:m, m] = wf
        Kb[m, :m] = wf
        self.Kb = Kb
        self.lu = sla.lu_factor(Kb)

    def solve(self, b):
        rhs = np.append(b[self.idx], 0.0)
        z = sla.lu_solve(self.lu, rhs)
        x = np.zeros_like(b)
        x[self.idx] = z[:-1]
        return x


class Hierarchy:
    """Levels n_l = m 2^l for l = coarse..fine (m macro cubes per axis)."""

    def __init__(self, dim, m, fine_level, coarse_level, inclusions, mu_table, form,
                 nu1=3, nu2=3, omega=OMEGA, coarse_mu='centroid', coarse_form=None, nu_inc=0,
                 mid_form=None, table=None, coarse_rhs_mod=False, bc='noslip', coarse_solver='direct',
                 minres_iters=30, cg_iters=5):
        """coarse_mu: 'centroid' rediscretises every level with the centroid
        rule; 'average' uses averaged_coarse_viscosity below the finest
        level (``table``: its table-size model, None = exact averages).
        mid_form: viscous form of the levels strictly between the finest and
        the coarsest (default: ``form``).  coarse_form: viscous form of the
        coarsest level (Sec. 5 swaps to the strain form on the coarse grid;
        default: the form of the levels above).  nu_inc: variable V-cycle
        (V_var of Sec. 5), nu_inc more pre- and post-smoothing steps per
        level below the finest.  coarse_rhs_mod: when the coarsest level's
        form differs from the one above it, its momentum right-hand side
        r_1 is replaced by r_1 + B^T M^-1 r_2 with M the lumped
        (1/mu)-weighted pressure mass (Sec. 5, coarse grid solver; the
        paper writes r_1 - B^T M^-1 r_2 for its opposite sign of B).
        bc: 'noslip' or 'freeslip' on every level (mesh.fixed_velocity).
        coarse_solver: 'direct' (bordered dense LU) or 'minres' (the
        block-diagonally preconditioned MINRES of Sec. 5, krylov.py, with
        minres_iters outer and cg_iters inner Jacobi-CG steps)."""
        self.dim = dim
        self.levels = {}
        self.P = {}
        mform = form if mid_form is None else mid_form
        cform = mform if coarse_form is None else coarse_form
        mu_f = imu_f = None
        for l in range(fine_level, coarse_level - 1, -1):
            n = m * 2 ** l
            f = form if l == fine_level else (cform if l == coarse_level else mform)
            if l == fine_level or coarse_mu == 'centroid':
                self.levels[l] = Level(dim, n, inclusions, mu_table, f, bc=bc)
                mu_f, imu_f = self.levels[l].disc.mu_e, self.levels[l].disc.imu_e
            else:
                mu_f, imu_f, mq, iq = averaged_coarse_viscosity(dim, n, mu_f, imu_f, list(mu_table),
                                                                table=table)
                self.levels[l] = Level(dim, n, inclusions, mu_table, f, mu_e=mq, imu_e=iq, bc=bc)
            if l > coarse_level:
                self.P[l] = prolongation(dim, m * 2 ** (l - 1))
        self.fine, self.coarse = fine_level, coarse_level
        if coarse_solver == 'direct':
            self.coarse_solver = CoarseSolver(self.levels[coarse_level])
        elif coarse_solver == 'minres':
            from . import krylov
            self.coarse_solver = krylov.MinresCoarseSolver(self.levels[coarse_level], minres_iters, cg_iters)
        else:
            raise ValueError(coarse_solver)
        self.nu1, self.nu2, self.omega, self.nu_inc = nu1, nu2, omega, nu_inc
        self.coarse_rhs_mod = (coarse_rhs_mod and fine_level > coarse_level and
                               self.levels[coarse_level].form != self.levels[coarse_level + 1].form)

    def prolong(self, l, xc):
        P, dim = self.P[l], self.dim
        Nc = P.shape[1]
        return np.concatenate([P @ xc[k * Nc:(k + 1) * Nc] for k in range(dim + 1)])

    def restrict(self, l, rf):
        P, dim = self.P[l], self.dim
        Nf, Nc = P.shape
        rc = np.concatenate([P.T @ rf[k * Nf:(k + 1) * Nf] for k in range(dim + 1)])
        return rc * self.levels[l - 1].free

    def vcycle(self, l, x, b):
        lv = self.levels[l]
        if l == self.coarse:
            if self.coarse_rhs_mod:
                N, d = lv.N, self.dim
                b = b.copy()
                b[:d * N] += lv.BT @ (b[d * N:] / lv.weights)
            return self.coarse_solver.solve(b)
        extra = self.nu_inc * (self.fine - l)
        x = smooth(lv, x, b, self.nu1 + extra, self.omega)
        r = residual(lv, x, b)
        ec = self.vcycle(l - 1, np.zeros(self.levels[l - 1].K.shape[0]), self.restrict(l, r))
        x = x + self.prolong(l, ec)
        return smooth(lv, x, b, self.nu2 + extra, self.omega)

    def solve(self, b, rtol=1e-8, maxit=100, x0=None):
        lv = self.levels[self.fine]
        x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
        nb = np.linalg.norm(b)
        hist = [np.linalg.norm(residual(lv, x, b)) / nb]
        while hist[-1] > rtol and len(hist) <= maxit:
            x = self.vcycle(self.fine, x, b)
            hist.append(np.linalg.norm(residual(lv, x, b)) / nb)
        return x, np.array(hist)

    def rate_history(self, x0, iters):
        """Residual reduction of every cycle of the stationary iteration on
        the homogeneous problem K x = 0 from x0, rescaling the iterate every
        step (the measurement of Sec. 5); the last entries approach the
        asymptotic rate."""
        lv = self.levels[self.fine]
        x = np.array(x0, dtype=np.float64) * lv.free
        b = np.zeros_like(x)
        N = lv.N
        rates = []
        for _ in range(iters):
            r0 = np.linalg.norm(lv.K @ x)
            x = self.vcycle(self.fine, x, b)
            # the constant pressure is in the kernel of K; remove it so that
            # the rescaling does not let it grow without bound
            x[self.dim * N:] -= np.dot(lv.weights, x[self.dim * N:]) / lv.weights.sum()
            r1 = np.linalg.norm(lv.K @ x)
            rates.append(r1 / r0)
            x /= r1
        return np.array(rates)

    def asymptotic_rate(self, iters=200, seed=0):
        """Residual reduction per cycle on the homogeneous problem after
        ``iters`` cycles, rescaling the iterate every step (Sec. 5)."""
        lv = self.levels[self.fine]
        rng = np.random.default_rng(seed)
        return self.rate_history(rng.uniform(-1, 1, lv.K.shape[0]), iters)[-1]


def direct_solve(lv, b):
    """Reference x* = K^+ b on the free dofs, pressure normalised."""
    cs = CoarseSolver(lv)
    return cs.solve(b)


def fgmres(apply_K, precond, b, rtol=1e-8, restart=40, maxit=200, x0=None):
    """Right-preconditioned flexible GMRES (Saad, SIAM J. Sci. Comput. 14,
    1993) in FP64 with modified Gram-Schmidt and Givens rotations.

    Used as the outer iteration when the stationary V-cycle does not
    contract (viscosity contrasts far above the paper's tests; Sec. 5 only
    reports contrast 10).  ``precond`` is one V-cycle from a zero guess.
    Returns x and the relative residual history (one entry per iteration,
    the first being the initial residual)."""
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    nb = np.linalg.norm(b)
    r = b - apply_K(x)
    beta = np.linalg.norm(r)
    hist = [beta / nb]
    its = 0
    while hist[-1] > rtol and its < maxit:
        V = [r / beta]
        Z = []
        H = np.zeros((restart + 1, restart))
        cs, sn = np.zeros(restart), np.zeros(restart)
        g = np.zeros(restart + 1)
        g[0] = beta
        j = 0
        while j < restart and its < maxit:
            z = precond(V[j])
            Z.append(z)
            w = apply_K(z)
            for i in range(j + 1):
                H[i, j] = np.dot(V[i], w)
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            V.append(w / H[j + 1, j] if H[j + 1, j] > 0 else w)
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = np.hypot(H[j, j], H[j + 1, j])
            cs[j], sn[j] = H[j, j] / den, H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            j += 1
            its += 1
            hist.append(abs(g[j]) / nb)
            if hist[-1] <= rtol:
                break
        y = np.linalg.solve(np.triu(H[:j, :j]), g[:j])
        for i in range(j):
            x = x + y[i] * Z[i]
        r = b - apply_K(x)
        beta = np.linalg.norm(r)
        hist[-1] = beta / nb
    return x, np.array(hist)


def stationary_cycles(hier, r, cycles=1):
    """z after ``cycles`` steps of the stationary V-cycle iteration
    z <- V(z; r) on K z = r from z = 0 (the preconditioner of the outer
    Krylov iteration; one step is the plain V-cycle of Sec. 5)."""
    z = np.zeros_like(r)
    for _ in range(cycles):
        z = hier.vcycle(hier.fine, z, r)
    return z


def solve_fgmres(hier, b, rtol=1e-8, restart=40, maxit=200, cycles=1):
    lv = hier.levels[hier.fine]
    return fgmres(lambda v: lv.K @ v,
                  lambda r: stationary_cycles(hier, r, cycles),
                  b, rtol=rtol, restart=restart, maxit=maxit)
