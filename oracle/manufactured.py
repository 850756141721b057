"""Manufactured 2D interface solution for the convergence pin.

The paper's only closed-form interface solution is 3D Couette flow (Sec. 4);
the 2D workload needs one with the interface x = 1/2 and mu = mu_1 (x < 1/2),
mu_2 (x > 1/2).  Reading taken: with the stream function

    psi(x, y) = (x - 1/2)^2 x^2 (1 - x)^2 y^2 (1 - y)^2

set u = curl psi / mu_i = (d_y psi, -d_x psi) / mu_i in Omega_i and
p = cos(pi x) cos(pi y).  Then div u = 0, u = 0 on the boundary, u is
continuous across x = 1/2 (psi has a double root there), mu_i grad u =
grad curl psi is smooth so the stress jump of eq. stokes-strong-interface
vanishes, and f = -mu_i Laplace u + grad p = -Laplace curl psi + grad p is
smooth and independent of mu.  Derivatives are taken symbolically.
"""
import numpy as np
import sympy as sy

_x, _y = sy.symbols('x y', real=True)
_psi = (_x - sy.Rational(1, 2)) ** 2 * _x ** 2 * (1 - _x) ** 2 * _y ** 2 * (1 - _y) ** 2
_p = sy.cos(sy.pi * _x) * sy.cos(sy.pi * _y)
_curl = (sy.diff(_psi, _y), -sy.diff(_psi, _x))
_lap = lambda e: sy.diff(e, _x, 2) + sy.diff(e, _y, 2)
_f = (sy.expand(-_lap(_curl[0]) + sy.diff(_p, _x)),
      sy.expand(-_lap(_curl[1]) + sy.diff(_p, _y)))

_curl_fn = sy.lambdify((_x, _y), _curl, 'numpy')
_p_fn = sy.lambdify((_x, _y), _p, 'numpy')
_f_fn = sy.lambdify((_x, _y), _f, 'numpy')


def symbols():
    """(x, y, psi, p, curl psi, f) as sympy expressions (for the pins)."""
    return _x, _y, _psi, _p, _curl, _f


def velocity(xy, mu1, mu2):
    x, y = xy[:, 0], xy[:, 1]
    c = np.array(_curl_fn(x, y), dtype=np.float64)
    mu = np.where(x < 0.5, mu1, mu2)
    return (c / mu).T


def pressure(xy):
    return np.asarray(_p_fn(xy[:, 0], xy[:, 1]), dtype=np.float64) * np.ones(len(xy))


def force(xy):
    f = _f_fn(xy[:, 0], xy[:, 1])
    return np.stack([np.asarray(fi, dtype=np.float64) * np.ones(len(xy)) for fi in f], axis=1)
