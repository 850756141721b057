"""P1 element matrices, written from the bilinear forms of the paper.

Notation: an element T has vertices x_0..x_d; lambda_i are its barycentric
coordinates (the P1 hat functions restricted to T), g_i = grad lambda_i and
|T| its volume.  A vector basis function is phi_i e_k (vertex i, component
k); its gradient is the d x d matrix (grad u)_{ab} = d u_a / d x_b =
delta_{ak} g_i[b].

Local degrees of freedom of the velocity are ordered a = i * d + k.  All
local matrices are indexed [test, trial]: entry (j l, i k) is
form(phi_i e_k, phi_j e_l).
"""
import math

import numpy as np

# Stabilisation constant of the P1-P1 pressure block.  The paper only names
# the Brezzi-Pitkaranta stabilisation for its equal-order runs (Sec. 4,
# opening paragraph) and gives no formula.  The reading taken here is
#     c(p, q) = sum_T  beta * h^2 / mu_T * (grad p, grad q)_T,
# beta = 1/12, h = axis edge length 1/n; the 1/mu scaling follows the
# pressure norm (p/(2 mu), q) of Sec. 3 and the 1/(2 mu_i) of eq. stabc.
STAB_BETA = 1.0 / 12.0


def simplex_geometry(X):
    """Barycentric gradients and volumes of a batch of simplices.

    X: (E, d+1, d) vertex coordinates.  With M = [1 | X] (rows [1, x_i]),
    lambda(x) = [1, x] M^{-1}, so column i of M^{-1} holds lambda_i's
    coefficients and rows 1..d of that column its gradient.
    Returns G (E, d+1, d) with G[e, i] = grad lambda_i, and vol (E,).
    """
    X = np.asarray(X, dtype=np.float64)
    E, dp1, d = X.shape
    M = np.concatenate([np.ones((E, dp1, 1)), X], axis=2)
    Minv = np.linalg.inv(M)
    G = np.transpose(Minv[:, 1:, :], (0, 2, 1))
    vol = np.abs(np.linalg.det(M)) / math.factorial(d)
    return G, vol


def basis_gradients(G):
    """grad(phi_i e_k) for all local velocity dofs: (E, (d+1) d, d, d)."""
    E, dp1, d = G.shape
    Gr = np.zeros((E, dp1 * d, d, d))
    for i in range(dp1):
        for k in range(d):
            Gr[:, i * d + k, k, :] = G[:, i, :]
    return Gr


def viscous_element_matrices(G, vol, mu, form):
    """Local velocity matrices of one of the three viscous forms.

    form 'lap' : (mu grad u, grad v)                    gradient form (Sec. 1)
    form 'sym' : (2 mu sym grad u, sym grad v)          eq. standard
    form 'div' : (mu div u, div v)
    form 'tr'  : a_sym - (mu div u, div v)               eq. newbil
    Each is integrated exactly: the integrands are constant on T.
    Returns (E, (d+1) d, (d+1) d) indexed [test, trial].
    """
    Gr = basis_gradients(G)
    w = (mu * vol)[:, None, None]
    if form == 'lap':
        return w * np.einsum('eiab,ejab->eji', Gr, Gr)
    sym = 0.5 * (Gr + np.transpose(Gr, (0, 1, 3, 2)))
    div = np.trace(Gr, axis1=2, axis2=3)
    a_sym = 2.0 * w * np.einsum('eiab,ejab->eji', sym, sym)
    a_div = w * np.einsum('ei,ej->eji', div, div)
    if form == 'sym':
        return a_sym
    if form == 'div':
        return a_div
    if form == 'tr':
        return a_sym - a_div
    raise ValueError(form)


def divergence_element_matrices(G, vol):
    """b(v, q) = -(div v, q) of eq. weaks with P1 pressure q = lambda_j.

    div(phi_i e_k) = g_i[k] is constant on T and int_T lambda_j = |T|/(d+1).
    Returns (E, d+1, (d+1) d): rows = pressure test function j,
    columns = velocity trial dof (i, k).
    """
    E, dp1, d = G.shape
    Gr = basis_gradients(G)
    div = np.trace(Gr, axis1=2, axis2=3)              # (E, (d+1) d)
    int_q = vol / dp1                                 # (E,)
    return -int_q[:, None, None] * np.ones((1, dp1, 1)) * div[:, None, :]


def stabilisation_element_matrices(G, vol, mu, h, beta=STAB_BETA):
    """c(p, q) restricted to T: beta h^2 / mu_T * (grad p, grad q)_T."""
    w = (beta * h * h / mu * vol)[:, None, None]
    return w * np.einsum('eia,eja->eji', G, G)


def mass_element_matrices(vol, d):
    """P1 mass matrix: int_T lambda_i lambda_j = |T| (1 + delta_ij) / ((d+1)(d+2))."""
    dp1 = d + 1
    base = (np.ones((dp1, dp1)) + np.eye(dp1)) / (dp1 * (dp1 + 1))
    return vol[:, None, None] * base[None]
