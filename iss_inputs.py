"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the
benchmark.  This module holds workload descriptions and random numbers only;
it contains none of the method's arithmetic.

Workloads (synthetic stand-ins for the paper's inclusion problems; the paper
times its own viscosity-columns problem, Sec. 4-5):

  square_split_2d  unit square, mu = 10 for x < 0.5 and 1 elsewhere,
                   2-triangle macro mesh refined 6 times (65 x 65 vertices),
                   coarsest level 3 (9 x 9)
  sphere_3d        unit cube, 6-tet macro mesh refined 6 times (65^3),
                   one sphere c = (0.5, 0.5, 0.5), r = 0.25, mu = 1000 inside,
                   buoyancy rho = 1 inside, coarsest level 3 (9^3)
  sinker_3d        unit cube as 2 x 2 x 2 macro cubes (48 tets) refined 7
                   times (257^3), 8 seeded spheres with centres
                   U[0.15, 0.85]^3 and radii U[0.05, 0.15], mu = 1e4 inside,
                   buoyancy inside, coarsest level 2 (9^3)
  learned_3d       unit cube refined 6 times (65^3), 1..16 seeded spheres
                   with centres U[0.2, 0.8]^3, radii U[0.05, 0.2] and one
                   contrast 10^U[1, 4] per problem
"""
import numpy as np

HALFSPACE, SPHERE, BOX = 'halfspace', 'sphere', 'box'


def _sphere(c, r, phase=1):
    return {'kind': SPHERE, 'center': tuple(float(v) for v in c), 'radius': float(r), 'phase': phase}


def workload(name, seed=0, levels=None):
    """Return a dict describing one workload.

    keys: dim, macro (cubes per axis), levels (refinements), coarse (coarsest
    level), n (cells per axis on the finest level), inclusions, mu (viscosity
    per phase, phase 0 = background), buoyant (phases with rho = 1)."""
    if name == 'square_split_2d':
        w = dict(dim=2, macro=1, levels=6, coarse=3,
                 inclusions=[{'kind': HALFSPACE, 'axis': 0, 'threshold': 0.5, 'phase': 1}],
                 mu=[1.0, 10.0], buoyant=[])
    elif name == 'sphere_3d':
        w = dict(dim=3, macro=1, levels=6, coarse=3,
                 inclusions=[_sphere((0.5, 0.5, 0.5), 0.25)],
                 mu=[1.0, 1000.0], buoyant=[1])
    elif name == 'sinker_3d':
        rng = np.random.default_rng(seed)
        centres = rng.uniform(0.15, 0.85, (8, 3))
        radii = rng.uniform(0.05, 0.15, 8)
        w = dict(dim=3, macro=2, levels=7, coarse=2,
                 inclusions=[_sphere(c, r) for c, r in zip(centres, radii)],
                 mu=[1.0, 1.0e4], buoyant=[1])
    elif name == 'columns_3d':
        # viscosity columns: the unit cube as 4^3 macro cubes, mu 10 in the
        # columns (0, 1/4)^2 x (0, 1) and (3/4, 1)^2 x (0, 1), mu 1 elsewhere,
        # free-slip on the whole boundary, forced by column_force below
        w = dict(dim=3, macro=4, levels=6, coarse=1,
                 inclusions=[{'kind': BOX, 'lo': (0.0, 0.0, 0.0), 'hi': (0.25, 0.25, 1.0), 'phase': 1},
                             {'kind': BOX, 'lo': (0.75, 0.75, 0.0), 'hi': (1.0, 1.0, 1.0), 'phase': 1}],
                 mu=[1.0, 10.0], buoyant=[], bc='freeslip', force='columns')
    elif name == 'learned_3d':
        rng = np.random.default_rng(seed)
        k = int(rng.integers(1, 17))
        centres = rng.uniform(0.2, 0.8, (k, 3))
        radii = rng.uniform(0.05, 0.2, k)
        contrast = 10.0 ** rng.uniform(1.0, 4.0)
        w = dict(dim=3, macro=1, levels=6, coarse=3,
                 inclusions=[_sphere(c, r) for c, r in zip(centres, radii)],
                 mu=[1.0, float(contrast)], buoyant=[1])
    else:
        raise KeyError(name)
    if levels is not None:
        w['levels'] = levels
    w['n'] = w['macro'] * 2 ** w['levels']
    w['name'] = name
    return w


def interior_mask(dim, n):
    """True for lattice vertices off the boundary of the unit cube/square
    (vertex v = i + (n+1) (j + (n+1) k), x fastest)."""
    idx = np.indices((n + 1,) * dim).reshape(dim, -1)[::-1]   # row 0 = i (x)
    return np.all((idx > 0) & (idx < n), axis=0)


def velocity_mask(dim, n, k, bc='noslip'):
    """1 where velocity component k is an unknown: interior vertices for
    'noslip'; for 'freeslip' every vertex off the faces x_k = 0, 1."""
    if bc == 'noslip':
        return interior_mask(dim, n)
    idx = np.indices((n + 1,) * dim).reshape(dim, -1)[::-1]
    return (idx[k] > 0) & (idx[k] < n)


def random_rhs(dim, n, seed, bc='noslip'):
    """b = (f, g) with f ~ U[-1, 1] on velocity entries that are unknowns,
    zero on fixed ones, and g = 0.  Field-major [f_1..f_d | g]."""
    rng = np.random.default_rng(seed)
    N = (n + 1) ** dim
    b = np.zeros((dim + 1) * N)
    for k in range(dim):
        b[k * N:(k + 1) * N] = rng.uniform(-1.0, 1.0, N) * velocity_mask(dim, n, k, bc)
    return b


def random_vector(dim, n, seed, zero_dirichlet=True, bc='noslip'):
    """x ~ U[-1, 1] on every entry; fixed velocity entries are zero when
    zero_dirichlet is set (the operators assume that)."""
    rng = np.random.default_rng(seed)
    N = (n + 1) ** dim
    x = rng.uniform(-1.0, 1.0, (dim + 1) * N)
    if zero_dirichlet:
        for k in range(dim):
            x[k * N:(k + 1) * N] *= velocity_mask(dim, n, k, bc)
    return x


def column_force(dim, n):
    """Nodal values (d fields of N) of the body force of the viscosity
    layers and columns, f = (0, 0, -cos(2 pi x) cos(2 pi y) sin(pi z)) in 3D
    (2D: f = (0, -cos(2 pi x) sin(pi y)))."""
    idx = np.indices((n + 1,) * dim).reshape(dim, -1)[::-1] / n
    f = np.zeros((dim, idx.shape[1]))
    if dim == 3:
        f[2] = -np.cos(2 * np.pi * idx[0]) * np.cos(2 * np.pi * idx[1]) * np.sin(np.pi * idx[2])
    else:
        f[1] = -np.cos(2 * np.pi * idx[0]) * np.sin(np.pi * idx[1])
    return f


def sample_vertices(dim, n, count, seed):
    rng = np.random.default_rng(seed)
    return np.unique(rng.integers(0, (n + 1) ** dim, count))
