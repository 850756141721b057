"""Kuhn lattices: vertices and simplices of uniformly refined cube/square meshes.

The paper's multigrid runs on block-structured meshes: an unstructured macro
mesh whose elements are refined uniformly (Sec. 2.2, the stencil discussion;
Sec. 5, HHG).  The test meshes are cubes split into six tetrahedra (Sec. 4,
viscosity layers) refined with Bey's rule (Sec. 3, remark on Bey-refined
meshes).  The resulting fine mesh is the Kuhn (Freudenthal) lattice: every
lattice cell is split into the d! simplices

    x0, x0 + e_pi(0), x0 + e_pi(0) + e_pi(1), ..., x0 + (1,...,1)

one per permutation pi.  In 2D this is the split of each square along its
(0,0)-(1,1) diagonal.  ``bey_refine`` builds the same element set by
recursive refinement of the macro elements so that a test can check that
claim instead of assuming it.

Vertex numbering (shared by every vector in the project): lattice index
(i, j[, k]) with 0 <= i, j, k <= n maps to v = i + (n+1) * (j + (n+1) * k),
x fastest.  Coordinates are (i, j, k) / n on the unit cube.
"""
import itertools

import numpy as np


def num_vertices(dim, n):
    return (n + 1) ** dim


def vertex_index(dim, n, ijk):
    """Linear vertex id of integer lattice coordinates ``ijk`` (..., dim)."""
    ijk = np.asarray(ijk)
    n1 = n + 1
    v = ijk[..., 0].astype(np.int64)
    stride = n1
    for a in range(1, dim):
        v = v + stride * ijk[..., a]
        stride *= n1
    return v


def vertex_ijk(dim, n):
    """Integer lattice coordinates of every vertex, shape (N, dim)."""
    n1 = n + 1
    v = np.arange(n1 ** dim, dtype=np.int64)
    out = np.empty((v.size, dim), dtype=np.int64)
    rem = v
    for a in range(dim):
        out[:, a] = rem % n1
        rem = rem // n1
    return out


def vertex_coords(dim, n):
    return vertex_ijk(dim, n).astype(np.float64) / n


def boundary_mask(dim, n):
    """True for vertices on the boundary of the unit cube / square."""
    ijk = vertex_ijk(dim, n)
    return np.any((ijk == 0) | (ijk == n), axis=1)


def fixed_velocity(dim, n, bc='noslip'):
    """Velocity components held at zero, shape (dim, N) bool (eq. boundary).

    'noslip': homogeneous Dirichlet, every component of every boundary
    vertex.  'freeslip': u . n = 0 on the faces of the unit cube / square,
    i.e. component k of a vertex on a face with normal e_k (i_k = 0 or n);
    the tangential components there are unknowns, and the zero tangential
    traction is the natural condition of the weak form (no boundary term).
    A vertex on an edge or corner has every normal of its faces fixed."""
    ijk = vertex_ijk(dim, n)
    on_face = (ijk == 0) | (ijk == n)                 # (N, dim)
    if bc == 'noslip':
        return np.repeat(np.any(on_face, axis=1)[None, :], dim, axis=0)
    if bc == 'freeslip':
        return on_face.T.copy()
    raise ValueError(bc)


def kuhn_offsets(dim):
    """The d! simplices of the unit cell as integer vertex offsets.

    Returns an array (d!, d+1, dim): simplex s has vertices
    0, e_pi(0), e_pi(0)+e_pi(1), ..., (1..1) for the s-th permutation pi.
    """
    simplices = []
    for perm in itertools.permutations(range(dim)):
        verts = [np.zeros(dim, dtype=np.int64)]
        for a in perm:
            nxt = verts[-1].copy()
            nxt[a] += 1
            verts.append(nxt)
        simplices.append(np.stack(verts))
    return np.stack(simplices)


def kuhn_elements(dim, n, cells=None):
    """Elements of the Kuhn lattice with n cells per axis.

    ``cells`` optionally restricts to a list of cell origins (M, dim); by
    default every cell of [0, n)^dim is used.  Returns int64 array
    (E, dim+1) of vertex ids, element e = cell c * d! + permutation s.
    """
    if cells is None:
        cells = vertex_ijk(dim, n - 1) if n >= 1 else np.zeros((0, dim), np.int64)
        # vertex_ijk(dim, n-1) enumerates 0..n-1 per axis = all cell origins
    cells = np.asarray(cells, dtype=np.int64)
    off = kuhn_offsets(dim)                      # (S, d+1, dim)
    ijk = cells[:, None, None, :] + off[None]     # (M, S, d+1, dim)
    return vertex_index(dim, n, ijk).reshape(-1, dim + 1)


def incident_elements(dim, n, verts):
    """Elements of the Kuhn lattice that contain at least one of ``verts``.

    Candidate cells are the 2^dim cells having the vertex as a corner; a
    candidate simplex is kept if it lies in the domain and contains the
    vertex.  Returns unique element vertex lists (E, dim+1).
    """
    verts = np.unique(np.asarray(verts, dtype=np.int64))
    n1 = n + 1
    ijk = np.empty((verts.size, dim), np.int64)
    rem = verts
    for a in range(dim):
        ijk[:, a] = rem % n1
        rem = rem // n1
    corner = np.array(list(itertools.product((0, 1), repeat=dim)), np.int64)
    cells = (ijk[:, None, :] - corner[None]).reshape(-1, dim)
    inside = np.all((cells >= 0) & (cells < n), axis=1)
    cells = np.unique(cells[inside], axis=0)
    elems = kuhn_elements(dim, n, cells)
    keep = np.isin(elems, verts).any(axis=1)
    return elems[keep]


def bey_refine(coords, elems):
    """One uniform refinement step.

    Tetrahedra follow Bey's ordered rule (J. Bey, Computing 55, 1995): with
    edge midpoints x_ab the children are the four corner tetrahedra and the
    inner octahedron cut along the x02-x13 diagonal, vertex order kept so
    that repeated refinement stays conforming.  Triangles are split into
    four (red refinement).  Coordinates are float arrays; midpoints are
    deduplicated by exact value (all coordinates are dyadic).
    """
    coords = [tuple(c) for c in coords]
    index = {c: i for i, c in enumerate(coords)}

    def mid(a, b):
        m = tuple((np.array(coords[a]) + np.array(coords[b])) / 2.0)
        if m not in index:
            index[m] = len(coords)
            coords.append(m)
        return index[m]

    out = []
    for el in elems:
        if len(el) == 3:
            x0, x1, x2 = el
            m01, m02, m12 = mid(x0, x1), mid(x0, x2), mid(x1, x2)
            out += [(x0, m01, m02), (m01, x1, m12), (m02, m12, x2), (m01, m12, m02)]
        else:
            x0, x1, x2, x3 = el
            m01, m02, m03 = mid(x0, x1), mid(x0, x2), mid(x0, x3)
            m12, m13, m23 = mid(x1, x2), mid(x1, x3), mid(x2, x3)
            out += [(x0, m01, m02, m03), (m01, x1, m12, m13),
                    (m02, m12, x2, m23), (m03, m13, m23, x3),
                    (m01, m02, m03, m13), (m01, m02, m12, m13),
                    (m02, m03, m13, m23), (m02, m12, m13, m23)]
    return np.array(coords), np.array(out, dtype=np.int64)


def macro_mesh(dim, m):
    """Macro mesh: the unit cube as m^3 cubes x 6 Kuhn tetrahedra (Sec. 4,
    viscosity layers, takes m = 4; here m is a parameter) or the unit square
    as m^2 squares x 2 triangles.  Returns (coords, elements)."""
    coords = vertex_coords(dim, m)
    return coords, kuhn_elements(dim, m)
