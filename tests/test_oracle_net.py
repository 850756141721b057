"""Pins of the FP64 band-correction network reference (CPU)."""
import numpy as np
import pytest
import scipy.ndimage as ndi

from oracle import net


def _rand_setup(n=6, seed=0, frac=0.6):
    rng = np.random.default_rng(seed)
    N = (n + 1) ** 3
    band = rng.uniform(size=N) < frac
    x = rng.normal(size=(net.C_IN, N)) * band
    w = rng.normal(size=net.num_params()) * 0.2
    return rng, N, band, x, w


def test_conv_is_cross_correlation():
    """Library pin: one channel pair of conv equals scipy.ndimage.correlate
    with zero padding (band = whole lattice)."""
    n = 7
    rng = np.random.default_rng(1)
    N = (n + 1) ** 3
    x = rng.normal(size=(1, N))
    W = rng.normal(size=(1, 1, 27))
    got = net.conv(x, W, n, np.ones(N, bool))[0].reshape(n + 1, n + 1, n + 1)
    k = np.zeros((3, 3, 3))
    for t, (dx, dy, dz) in enumerate(net.TAPS):
        k[dz + 1, dy + 1, dx + 1] = W[0, 0, t]
    ref = ndi.correlate(x[0].reshape(n + 1, n + 1, n + 1), k, mode="constant", cval=0.0)
    assert np.allclose(got, ref, rtol=1e-13, atol=1e-13)


def test_conv_transpose_is_adjoint():
    rng, N, band, x, w = _rand_setup()
    W = net.split_params(w)[1]
    xi = rng.normal(size=(16, N)) * band
    g = rng.normal(size=(16, N))
    lhs = np.sum(net.conv(xi, W, 6, band) * g)
    rhs = np.sum(xi * net.conv_transpose(g, W, 6, band))
    assert np.isclose(lhs, rhs, rtol=1e-12)


def test_backward_matches_finite_differences():
    rng, N, band, x, w = _rand_setup(n=4, seed=2)
    t = rng.normal(size=(net.C_OUT, N)) * band
    y, cache = net.forward(w, x, 4, band)
    loss, dy = net.mse(y, t, band)
    g = net.backward(w, cache, dy, 4, band)
    idx = rng.choice(w.size, 40, replace=False)
    h = 1e-6
    for i in idx:
        wp, wm = w.copy(), w.copy()
        wp[i] += h
        wm[i] -= h
        lp = net.mse(net.forward(wp, x, 4, band)[0], t, band)[0]
        lm = net.mse(net.forward(wm, x, 4, band)[0], t, band)[0]
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1e-3, abs(fd)) + 1e-9, (i, fd, g[i])


def test_positive_homogeneity():
    """No biases and ReLU: net(alpha x) = alpha net(x) for alpha > 0, so the
    correction scales linearly with the residual."""
    rng, N, band, x, w = _rand_setup(seed=3)
    y1, _ = net.forward(w, x, 6, band)
    y2, _ = net.forward(w, 3.5 * x, 6, band)
    assert np.allclose(y2, 3.5 * y1, rtol=1e-12, atol=1e-12)
    assert np.all(y1[:, ~band] == 0)


def test_band_is_chebyshev_dilation():
    n = 10
    N = (n + 1) ** 3
    iface = np.zeros(N, bool)
    v = 5 + 11 * (5 + 11 * 5)
    iface[v] = True
    b = net.band_mask(3, n, iface)
    assert b.sum() == 125
    ijk = np.stack(np.unravel_index(np.nonzero(b)[0], (11, 11, 11)))
    assert np.abs(ijk - 5).max() == 2


def test_adam_first_step():
    w = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 1e-3])
    w1, m, v = net.adam(w, g, np.zeros(3), np.zeros(3), 1, 0.01)
    assert np.allclose(w - w1, 0.01 * np.sign(g), rtol=1e-4)


def test_target_units_round_trip():
    """correction() inverts scale_targets() on the band (Jacobi units)."""
    n = 6
    N = (n + 1) ** 3
    rng = np.random.default_rng(5)
    band = rng.uniform(size=N) < 0.5
    lmu = rng.uniform(0, 4, N)
    e = rng.normal(size=4 * N)
    t = net.scale_targets(3, n, e, band, 0.7, 1.9, lmu, 1.0 / 12.0)
    c = net.correction(3, n, t, band, 0.7, 1.9, lmu, 1.0 / 12.0)
    mask = np.tile(band, 4)
    assert np.allclose(c[mask], e[mask], rtol=1e-12)
    assert np.all(c[~mask] == 0)
