"""Krylov coarse-grid solver of Sec. 5 (oracle; test infrastructure only).

Sec. 5 solves the coarse system with a minimal residual method (MINRES)
preconditioned block-diagonally: a Jacobi-preconditioned conjugate gradient
iteration stands in for the velocity block and the lumped mass matrix for
the pressure block, the coarse operator being the strain form (a_tr is
swapped out on the coarse grid because the preconditioner needs a positive
definite velocity block).

Readings taken where the paper is open:
  * the lumped pressure mass is the 1/mu-weighted one, w_j = sum_T |T| /
    ((d+1) mu_T) (the pressure norm of Sec. 3 and the weights of the space
    Q of Sec. 1);
  * the inner CG runs a fixed number of steps from zero, the outer MINRES a
    fixed number of steps from zero (the paper only asks that the stopping
    criteria keep the multigrid rates); zero CG steps means the Jacobi
    preconditioner of the velocity block alone;
  * the constant pressure, the null space of K, is removed from the
    right-hand side before the iteration (plain mean of the pressure
    residual) and the weighted pressure mean from the result, as the direct
    coarse solver does through its border.

MINRES follows Paige and Saunders (SIAM J. Numer. Anal. 12, 1975) in the
preconditioned form of Elman, Silvester and Wathen (Finite Elements and
Fast Iterative Solvers, 2005, Alg. 4.1); CG is Hestenes and Stiefel (1952)
with a diagonal preconditioner.
"""
import numpy as np


def jacobi_pcg(apply_A, diag, r, iters):
    """``iters`` steps of Jacobi-preconditioned CG on A u = r from u = 0.
    diag: the diagonal of A (entries <= 0 mark dofs that stay zero)."""
    inv = np.where(diag > 0, 1.0 / np.where(diag > 0, diag, 1.0), 0.0)
    u = np.zeros_like(r)
    res = r.copy()
    z = inv * res
    p = z.copy()
    rz = res @ z
    for _ in range(iters):
        if rz == 0.0:
            break
        q = apply_A(p)
        alpha = rz / (p @ q)
        u = u + alpha * p
        res = res - alpha * q
        z = inv * res
        rz_new = res @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
    return u


def minres(apply_K, apply_Pinv, b, iters):
    """``iters`` steps of preconditioned MINRES on K x = b from x = 0 (K
    symmetric, P symmetric positive definite).  Returns x and the
    preconditioned residual estimates |eta| after each step."""
    x = np.zeros_like(b)
    v_old = np.zeros_like(b)
    v = b.copy()
    z = apply_Pinv(v)
    gamma = np.sqrt(max(v @ z, 0.0))
    gamma_old = 1.0
    w_old = np.zeros_like(b)
    w = np.zeros_like(b)
    eta = gamma
    s_old = s = 0.0
    c_old = c = 1.0
    hist = []
    for _ in range(iters):
        if gamma == 0.0:
            break
        z = z / gamma
        q = apply_K(z)
        delta = q @ z
        v_new = q - (delta / gamma) * v - (gamma / gamma_old) * v_old
        z_new = apply_Pinv(v_new)
        gamma_new = np.sqrt(max(v_new @ z_new, 0.0))
        a0 = c * delta - c_old * s * gamma
        a1 = np.sqrt(a0 * a0 + gamma_new * gamma_new)
        a2 = s * delta + c_old * c * gamma
        a3 = s_old * gamma
        c_new, s_new = a0 / a1, gamma_new / a1
        w_new = (z - a3 * w_old - a2 * w) / a1
        x = x + (c_new * eta) * w_new
        eta = -s_new * eta
        hist.append(abs(eta))
        v_old, v = v, v_new
        z = z_new
        gamma_old, gamma = gamma, gamma_new
        w_old, w = w, w_new
        c_old, c = c, c_new
        s_old, s = s, s_new
    return x, np.array(hist)


class MinresCoarseSolver:
    """Block-diagonally preconditioned MINRES on the coarse level ``lv``
    (a multigrid.Level): P^-1 (r_u, r_p) = (CG_m(A; r_u), r_p / w)."""

    def __init__(self, lv, minres_iters=30, cg_iters=5):
        self.lv = lv
        self.minres_iters, self.cg_iters = minres_iters, cg_iters
        d, N = lv.dim, lv.N
        self.dN = d * N
        self.diagA = lv.A.diagonal() * lv.free[:d * N]

    def apply_Pinv(self, r):
        lv = self.lv
        out = np.empty_like(r)
        if self.cg_iters > 0:
            out[:self.dN] = jacobi_pcg(lambda u: lv.A @ u, self.diagA, r[:self.dN], self.cg_iters)
        else:
            # no CG step: the Jacobi preconditioner of the velocity block itself
            d = self.diagA
            out[:self.dN] = np.where(d > 0, r[:self.dN] / np.where(d > 0, d, 1.0), 0.0)
        out[self.dN:] = r[self.dN:] / lv.weights
        return out

    def solve(self, b):
        lv = self.lv
        b = b * lv.free
        b[self.dN:] -= b[self.dN:].mean()
        x, _ = minres(lambda v: lv.K @ v, self.apply_Pinv, b, self.minres_iters)
        p = x[self.dN:]
        p -= np.dot(lv.weights, p) / lv.weights.sum()
        return x
