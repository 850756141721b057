"""Pins of the oracle's coarse-grid Krylov solver (Sec. 5: block-diagonally
preconditioned MINRES with Jacobi-CG on the velocity block and the lumped
mass on the pressure block) against the defining minimisation properties,
checked by brute force over explicit Krylov bases (no GPU)."""
import numpy as np
import pytest

import iss_inputs
from oracle import krylov, multigrid as mg


def _krylov_basis(apply, r, k):
    V = [r]
    for _ in range(k - 1):
        V.append(apply(V[-1]))
    Q, _ = np.linalg.qr(np.array(V).T)
    return Q


@pytest.mark.parametrize("k", [1, 2, 3, 5, 8])
def test_pcg_minimises_the_energy_error(k):
    """After k steps from zero, Jacobi-PCG minimises ||u* - u||_A over
    u in D^-1 K_k(A D^-1, r) (Hestenes-Stiefel)."""
    rng = np.random.default_rng(1)
    n = 40
    G = rng.standard_normal((n, n))
    A = G @ G.T + n * np.eye(n) * rng.uniform(0.5, 2.0, n)
    d = np.diag(A).copy()
    r = rng.standard_normal(n)
    u = krylov.jacobi_pcg(lambda v: A @ v, d, r, k)
    us = np.linalg.solve(A, r)
    # basis of D^-1 K_k(A D^-1, r) = span{D^-1 r, (D^-1 A) D^-1 r, ...}
    Q = _krylov_basis(lambda v: (A @ v) / d, r / d, k)
    y = np.linalg.solve(Q.T @ A @ Q, Q.T @ r)
    ub = Q @ y
    assert np.linalg.norm(u - ub) <= 1e-9 * np.linalg.norm(us)
    if k == 8:
        full = krylov.jacobi_pcg(lambda v: A @ v, d, r, n)
        assert np.linalg.norm(full - us) <= 1e-8 * np.linalg.norm(us)


def test_pcg_keeps_masked_dofs_zero():
    rng = np.random.default_rng(2)
    n = 12
    G = rng.standard_normal((n, n))
    A = G @ G.T + n * np.eye(n)
    mask = np.ones(n, bool)
    mask[[0, 5]] = False
    Am = A * np.outer(mask, mask)
    d = np.diag(Am) * mask
    r = rng.standard_normal(n) * mask
    u = krylov.jacobi_pcg(lambda v: Am @ v, d, r, 6)
    assert np.all(u[~mask] == 0)


@pytest.mark.parametrize("k", [1, 2, 4, 7])
def test_minres_minimises_the_preconditioned_residual(k):
    """After k steps from zero, preconditioned MINRES minimises
    ||b - K x||_{P^-1} over x in K_k(P^-1 K, P^-1 b) (Paige-Saunders), for
    a symmetric indefinite K and an SPD diagonal P; and its |eta| estimate
    is that minimal residual norm."""
    rng = np.random.default_rng(3)
    n = 30
    G = rng.standard_normal((n, n))
    K = G + G.T + np.diag(rng.uniform(-3, 3, n))
    p = rng.uniform(0.5, 2.0, n)
    b = rng.standard_normal(n)
    x, hist = krylov.minres(lambda v: K @ v, lambda v: v / p, b, k)
    Q = _krylov_basis(lambda v: (K @ v) / p, b / p, k)
    # minimise (b - K Q y)^T P^-1 (b - K Q y)
    W = np.diag(1.0 / np.sqrt(p))
    y, *_ = np.linalg.lstsq(W @ K @ Q, W @ b, rcond=None)
    xb = Q @ y
    assert np.linalg.norm(x - xb) <= 1e-8 * max(1.0, np.linalg.norm(xb))
    res = b - K @ x
    assert abs(np.sqrt(res @ (res / p)) - hist[-1]) <= 1e-9 * np.sqrt(b @ (b / p))
    assert np.all(np.diff(hist) <= 1e-12)


def test_minres_reaches_the_solution():
    rng = np.random.default_rng(4)
    n = 25
    G = rng.standard_normal((n, n))
    K = G + G.T
    b = rng.standard_normal(n)
    x, _ = krylov.minres(lambda v: K @ v, lambda v: v, b, n)
    assert np.linalg.norm(K @ x - b) <= 1e-8 * np.linalg.norm(b)


def test_minres_coarse_solver_approaches_the_direct_solve():
    """On a Stokes coarse level (columns problem, free-slip, 9^3, strain
    form) the block-preconditioned MINRES error to the bordered direct solve
    falls with the iteration counts, and the MINRES coarse solver gives the
    same two-grid rate as the direct one once it is accurate enough."""
    w = iss_inputs.workload('columns_3d')
    lv = mg.Level(3, 8, w['inclusions'], w['mu'], 'strain', bc='freeslip')
    b = iss_inputs.random_rhs(3, 8, seed=5, bc='freeslip')
    b[3 * lv.N:] = np.random.default_rng(6).uniform(-1, 1, lv.N)
    # a consistent right-hand side (orthogonal to the constant pressure, the
    # null space of the symmetric K), as a restricted residual of a problem
    # with g = 0 is
    b[3 * lv.N:] -= b[3 * lv.N:].mean()
    xd = mg.direct_solve(lv, b)
    errs = []
    for it, cg in [(5, 2), (20, 5), (80, 20)]:
        x = krylov.MinresCoarseSolver(lv, it, cg).solve(b)
        errs.append(np.linalg.norm(x - xd) / np.linalg.norm(xd))
    assert errs[0] > errs[1] > errs[2] and errs[2] < 1e-3, errs

    def rate(**kw):
        H = mg.Hierarchy(3, 4, 2, 1, w['inclusions'], w['mu'], 'interface', nu1=3, nu2=3, nu_inc=2, omega=0.3,
                         coarse_mu='average', bc='freeslip', coarse_form='strain', coarse_rhs_mod=True, **kw)
        return H.asymptotic_rate(iters=30, seed=1)

    rd = rate()
    rm = rate(coarse_solver='minres', minres_iters=30, cg_iters=5)
    assert abs(rm - rd) < 0.02, (rm, rd)


def test_zero_cg_steps_is_the_jacobi_block():
    """With no CG step the velocity block of the preconditioner is the
    Jacobi diagonal of A (and the pressure block the lumped mass)."""
    w = iss_inputs.workload('columns_3d')
    lv = mg.Level(3, 4, w['inclusions'], w['mu'], 'strain', bc='freeslip')
    S = krylov.MinresCoarseSolver(lv, 5, 0)
    r = np.random.default_rng(7).uniform(-1, 1, lv.K.shape[0]) * lv.free
    out = S.apply_Pinv(r)
    dN = 3 * lv.N
    d = lv.A.diagonal()
    free = lv.free[:dN]
    assert np.allclose(out[:dN][free], r[:dN][free] / d[free], rtol=1e-15, atol=0)
    assert np.all(out[:dN][~free] == 0)
    assert np.allclose(out[dN:], r[dN:] / lv.weights, rtol=1e-15, atol=0)
