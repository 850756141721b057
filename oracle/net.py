"""FP64 reference of the learned interface-band correction.

The correction network is not part of the paper; it is the learned
component added beside its smoother (a post-smoothing correction on the band
of vertices around the viscosity interface, where plain smoothing degrades,
cf. the interface discussion of Sec. 2.2).  Reading taken:

* band: lattice vertices within Chebyshev (index) distance 2 of an
  interface vertex of the finest level;
* input channels (8): the residual components r_1..r_d divided by the band
  RMS of the velocity residual s_u, r_p divided by the band RMS of the
  pressure residual s_p, log10(max incident viscosity) / 4, the interface
  flag, zero padding channels; every channel is zero off the band;
* network: three 3x3x3 convolutions 8 -> 16 -> 16 -> 4 with ReLU between
  them and no biases, zero padding off the band and outside the lattice
  (cross-correlation: out[v] = sum_tap w[tap] in[v + tap]);
* outputs are in Jacobi units: output channel c times s_u / (6 mu h)
  (velocity) or s_p mu / (6 beta h^3) (pressure), mu the largest incident
  viscosity, is the correction added to the iterate on the band;
* loss: mean squared error over band vertices and the 4 output channels,
  against the exact error in the same units (``mse``); the solver-side
  training objective, the residual left after the correction, reaches this
  module through ``backward`` with dL/dy supplied by the caller.

Everything here is plain numpy in FP64, written as direct loops over the 27
taps; the backward pass is derived by hand.
"""
import itertools

import numpy as np

C_IN, C_HID, C_OUT = 8, 16, 4
# taps are (dx, dy, dz) offsets in lattice index space, x fastest in the
# tap numbering: tap = (dx + 1) + 3 (dy + 1) + 9 (dz + 1)
TAPS = [np.array((dx, dy, dz)) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]

LAYERS = [(C_IN, C_HID), (C_HID, C_HID), (C_HID, C_OUT)]


def num_params():
    return sum(co * ci * 27 for ci, co in LAYERS)


def split_params(w):
    """Flat FP32/FP64 parameter vector -> [W1, W2, W3], W[co, ci, tap]."""
    out, o = [], 0
    for ci, co in LAYERS:
        n = co * ci * 27
        out.append(np.asarray(w[o:o + n], dtype=np.float64).reshape(co, ci, 27))
        o += n
    return out


def band_mask(dim, n, interface):
    """Vertices within Chebyshev distance 2 of an interface vertex."""
    shape = (n + 1,) * dim
    it = interface.reshape(shape[::-1])            # axes (z, y, x)
    out = np.zeros_like(it)
    for off in itertools.product(range(-2, 3), repeat=dim):
        src = [slice(max(0, -o), s - max(0, o)) for o, s in zip(off, it.shape)]
        dst = [slice(max(0, o), s - max(0, -o)) for o, s in zip(off, it.shape)]
        out[tuple(dst)] |= it[tuple(src)]
    return out.reshape(-1)


def shift(field, tap, n):
    """g[v] = field[v + tap] with zeros outside the lattice; field is a
    (n+1)^3 array flattened x fastest, or (..., N) with channels first."""
    f = field.reshape(field.shape[:-1] + (n + 1, n + 1, n + 1))    # (..., z, y, x)
    g = np.zeros_like(f)
    dx, dy, dz = tap
    sl_src, sl_dst = [], []
    for o, s in ((dz, n + 1), (dy, n + 1), (dx, n + 1)):
        sl_src.append(slice(max(0, o), s + min(0, o)))
        sl_dst.append(slice(max(0, -o), s + min(0, -o)))
    g[(Ellipsis,) + tuple(sl_dst)] = f[(Ellipsis,) + tuple(sl_src)]
    return g.reshape(field.shape)


def conv(x, W, n, band):
    """out[co, v] = sum_{ci, tap} W[co, ci, tap] x[ci, v + tap] on band
    vertices (zero elsewhere).  x: (ci, N)."""
    co = W.shape[0]
    out = np.zeros((co, x.shape[1]))
    for t, tap in enumerate(TAPS):
        xs = shift(x, tap, n)
        out += W[:, :, t] @ xs
    return out * band


def conv_transpose(g, W, n, band):
    """Gradient of conv with respect to its input: dx[ci, u] = sum_{co, tap}
    W[co, ci, tap] g[co, u - tap] (g zero off the band)."""
    ci = W.shape[1]
    out = np.zeros((ci, g.shape[1]))
    gb = g * band
    for t, tap in enumerate(TAPS):
        out += W[:, :, t].T @ shift(gb, -tap, n)
    return out


def conv_weight_grad(g, x, n, band):
    """dW[co, ci, tap] = sum_v g[co, v] x[ci, v + tap] over band vertices."""
    gb = g * band
    return np.stack([gb @ shift(x, tap, n).T for tap in TAPS], axis=2)


def forward(w, x, n, band):
    """Returns output (C_OUT, N) and the cache for backward."""
    W1, W2, W3 = split_params(w)
    z1 = conv(x, W1, n, band)
    a1 = np.maximum(z1, 0.0)
    z2 = conv(a1, W2, n, band)
    a2 = np.maximum(z2, 0.0)
    y = conv(a2, W3, n, band)
    return y, (x, z1, a1, z2, a2)


def mse(y, target, band):
    m = band.sum() * y.shape[0]
    d = (y - target) * band
    return float(np.sum(d * d) / m), 2.0 * d / m


def backward(w, cache, dy, n, band):
    """Gradient of a scalar loss with respect to the flat parameters, given
    dL/dy (C_OUT, N)."""
    W1, W2, W3 = split_params(w)
    x, z1, a1, z2, a2 = cache
    gW3 = conv_weight_grad(dy, a2, n, band)
    da2 = conv_transpose(dy, W3, n, band) * band
    dz2 = da2 * (z2 > 0)
    gW2 = conv_weight_grad(dz2, a1, n, band)
    da1 = conv_transpose(dz2, W2, n, band) * band
    dz1 = da1 * (z1 > 0)
    gW1 = conv_weight_grad(dz1, x, n, band)
    return np.concatenate([gW1.ravel(), gW2.ravel(), gW3.ravel()])


def features(dim, n, r, band, log_mu_max, interface):
    """Input channels from a residual r ((d+1) N, field-major) and the
    scales (s_u, s_p): band RMS of the velocity residual components and of
    the pressure residual (1 if zero)."""
    N = (n + 1) ** dim
    ru = r[:dim * N].reshape(dim, N)
    rp = r[dim * N:]
    nb = max(int(band.sum()), 1)
    s_u = np.sqrt(np.sum(ru[:, band] ** 2) / (dim * nb))
    s_p = np.sqrt(np.sum(rp[band] ** 2) / nb)
    s_u = s_u if s_u > 0 else 1.0
    s_p = s_p if s_p > 0 else 1.0
    x = np.zeros((C_IN, N))
    x[:dim] = ru / s_u
    x[dim] = rp / s_p
    x[4] = log_mu_max / 4.0
    x[5] = interface.astype(np.float64)
    return x * band, s_u, s_p


def diagonal_scales(n, log_mu_max, beta):
    """Jacobi units of the targets: the diagonal of the isoviscous 3D
    operator rows at viscosity mu = 10^log_mu_max, 6 mu h for a velocity
    component and 6 beta h^3 / mu for the pressure (reading taken for the
    output units of the network)."""
    h = 1.0 / n
    mu = 10.0 ** log_mu_max
    return 6.0 * mu * h, 6.0 * beta * h ** 3 / mu


def scale_targets(dim, n, e, band, s_u, s_p, log_mu_max, beta):
    N = (n + 1) ** dim
    du, dp = diagonal_scales(n, np.where(band, log_mu_max, 0.0), beta)
    t = np.zeros((C_OUT, N))
    t[:dim] = e[:dim * N].reshape(dim, N) * du / s_u
    t[dim] = e[dim * N:] * dp / s_p
    return t * band


def correction(dim, n, y, band, s_u, s_p, log_mu_max, beta):
    """Network output back to a (d+1) N correction vector."""
    N = (n + 1) ** dim
    du, dp = diagonal_scales(n, np.where(band, log_mu_max, 0.0), beta)
    c = np.zeros((dim + 1) * N)
    c[:dim * N] = (y[:dim] * band * s_u / du).ravel()
    c[dim * N:] = y[dim] * band * s_p / dp
    return c


def adam(w, g, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba 2015) with bias correction."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v
