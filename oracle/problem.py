"""Problem data: element viscosity, interface vertices, right-hand sides.

Viscosity is piecewise constant (Sec. 1).  The inclusion geometries of the
workloads are spheres and half-spaces that the meshes do not resolve, the
situation of the remark closing Sec. 2.2: shape functions whose support
meets more than one viscosity are the interface ones.

Reading taken for unresolved geometry: an element takes the viscosity of
the first inclusion (list order) whose open region contains its centroid,
else the background viscosity (phase 0).  A vertex is an interface vertex
when the viscosities of its incident elements are not all equal (compared
as numbers, so two phases with equal viscosity do not make an interface).
"""
import numpy as np

from . import fem, mesh


def element_phase(dim, n, elems, inclusions):
    """Phase of each element by the centroid rule.

    inclusions: list of dicts {'kind': 'sphere', 'center': c, 'radius': r,
    'phase': p} or {'kind': 'halfspace', 'axis': a, 'threshold': t,
    'phase': p} (region x_a < t) or {'kind': 'box', 'lo': l, 'hi': h,
    'phase': p} (region l_a < x_a < h_a on every axis).  Strict
    inequalities: a centroid exactly on a sphere, plane or box face counts as
    outside.
    """
    X = mesh.vertex_coords(dim, n)[elems]            # (E, d+1, d)
    cen = X.mean(axis=1)
    phase = np.zeros(len(elems), dtype=np.int64)
    assigned = np.zeros(len(elems), dtype=bool)
    for inc in inclusions:
        if inc['kind'] == 'sphere':
            c = np.asarray(inc['center'], dtype=np.float64)[:dim]
            inside = np.sum((cen - c) ** 2, axis=1) < inc['radius'] ** 2
        elif inc['kind'] == 'halfspace':
            inside = cen[:, inc['axis']] < inc['threshold']
        elif inc['kind'] == 'box':
            lo = np.asarray(inc['lo'], dtype=np.float64)[:dim]
            hi = np.asarray(inc['hi'], dtype=np.float64)[:dim]
            inside = np.all((cen > lo) & (cen < hi), axis=1)
        else:
            raise ValueError(inc['kind'])
        new = inside & ~assigned
        phase[new] = inc['phase']
        assigned |= inside
    return phase


def element_mu(dim, n, elems, inclusions, mu_table):
    return np.asarray(mu_table, dtype=np.float64)[element_phase(dim, n, elems, inclusions)]


def interface_vertices(dim, n, elems, mu_e):
    """Boolean mask over vertices: incident element viscosities differ."""
    N = mesh.num_vertices(dim, n)
    lo = np.full(N, np.inf)
    hi = np.full(N, -np.inf)
    for a in range(dim + 1):
        np.minimum.at(lo, elems[:, a], mu_e)
        np.maximum.at(hi, elems[:, a], mu_e)
    return hi > lo


def vertex_phase(dim, n, elems, phase_e):
    """Phase of the incident elements of each vertex (any one of them)."""
    N = mesh.num_vertices(dim, n)
    out = np.zeros(N, dtype=np.int64)
    for a in range(dim + 1):
        out[elems[:, a]] = phase_e
    return out


def pressure_weights(dim, n, elems, mu_e):
    """w_j = int mu^{-1} lambda_j: the weights of the pressure space
    Q = {q : int mu^{-1} q = 0} of Sec. 1, for P1 pressure."""
    X = mesh.vertex_coords(dim, n)[elems]
    _, vol = fem.simplex_geometry(X)
    N = mesh.num_vertices(dim, n)
    w = np.zeros(N)
    for a in range(dim + 1):
        np.add.at(w, elems[:, a], vol / ((dim + 1) * mu_e))
    return w


def normalise_pressure(x, dim, n, weights):
    """Shift the pressure block so that sum_j w_j p_j = 0 (Sec. 1, Q)."""
    N = mesh.num_vertices(dim, n)
    y = np.array(x, dtype=np.float64, copy=True)
    p = y[dim * N:]
    p -= np.dot(weights, p) / np.sum(weights)
    return y


def rhs_buoyancy(dim, n, elems, phase_e, buoyant_phases, rho=1.0):
    """Load vector of the body force f = (0, .., 0, -rho) on elements of the
    buoyant phases: <f, lambda_j e_d> = -sum_{T ni j} rho |T| / (d+1).
    Pressure rows are zero (g = 0, Sec. 5 system)."""
    N = mesh.num_vertices(dim, n)
    X = mesh.vertex_coords(dim, n)[elems]
    _, vol = fem.simplex_geometry(X)
    dens = np.where(np.isin(phase_e, list(buoyant_phases)), rho, 0.0)
    b = np.zeros((dim + 1) * N)
    comp = (dim - 1) * N
    for a in range(dim + 1):
        np.add.at(b, comp + elems[:, a], -dens * vol / (dim + 1))
    return b


def rhs_from_nodal_force(dim, n, elems, f_nodal):
    """Consistent load of the P1 interpolant of a force: b_k = M f_k.

    f_nodal: (N, d) nodal values.  Pressure rows zero."""
    N = mesh.num_vertices(dim, n)
    X = mesh.vertex_coords(dim, n)[elems]
    _, vol = fem.simplex_geometry(X)
    Me = fem.mass_element_matrices(vol, dim)
    b = np.zeros((dim + 1) * N)
    for k in range(dim):
        fk = f_nodal[:, k][elems]                        # (E, d+1)
        contrib = np.einsum('eji,ei->ej', Me, fk)
        np.add.at(b, k * N + elems.ravel(), contrib.ravel())
    return b
