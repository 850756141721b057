"""GPU parity of the learned band-correction network (BF16 MFMA implicit
GEMM, FP32 accumulation) against the FP64 oracle.

Tolerances: scales (FP64) 1e-12; forward outputs entry by entry within the
BF16 rounding bound 9u A_3 (u = 2^-8, A_3 the convolution of magnitudes),
band-edge vertices included, and 2e-2 relative in the 2-norm over the band;
weight gradients entry by entry within 16u of the backward pass of
magnitudes, and 3e-2 relative in the 2-norm; Adam (FP32 vs FP64) 1e-5."""
import numpy as np
import pytest

import iss_inputs
from oracle import assemble, net as onet, problem as oprob
from tests.gpu_common import gpu_problem, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup():
    import torch
    from paper_1604_07994_amd.binding import BandNet
    w = iss_inputs.workload("learned_3d", seed=3, levels=4)
    P = gpu_problem(w, outer="fgmres", omega=0.6, restart=60, coarse_mu="average", coarse_form="strain")
    N = (w["n"] + 1) ** 3
    D = assemble.Discretisation(3, w["n"], w["inclusions"], w["mu"])
    band = onet.band_mask(3, w["n"], D.interface)
    lmu = np.full(N, -np.inf)
    np.maximum.at(lmu, D.elems.ravel(), np.repeat(np.log10(D.mu_e), 4))
    net = BandNet(P)
    rng = np.random.default_rng(7)
    wts = (rng.normal(size=onet.num_params()) * 0.15).astype(np.float32)
    net.set_weights(torch.from_numpy(wts).cuda())
    yield w, P, D, band, lmu, net, wts
    net.close()
    P.close()


def test_band_matches_oracle(setup):
    w, P, D, band, lmu, net, wts = setup
    assert np.array_equal(np.sort(net.band()), np.nonzero(band)[0])


def _oracle_forward(w, D, band, lmu, wts, r):
    x, su, sp = onet.features(3, w["n"], r, band, lmu, D.interface)
    y, cache = onet.forward(wts.astype(np.float64), x, w["n"], band)
    return x, su, sp, y, cache


def test_forward_parity(setup):
    import torch
    w, P, D, band, lmu, net, wts = setup
    r = iss_inputs.random_vector(3, w["n"], seed=8)
    su, sp = net.features(to_dev(r))
    y = torch.empty(net.band_size * 4, dtype=torch.float32, device="cuda")
    net.forward(y)
    x, osu, osp, oy, _ = _oracle_forward(w, D, band, lmu, wts, r)
    assert np.isclose(su, osu, rtol=1e-12) and np.isclose(sp, osp, rtol=1e-12)
    ref = oy[:, band].T                           # (M, 4) in band order
    got = to_host(y).reshape(-1, 4)
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    assert err < 2e-2, err


U_BF16 = 2.0 ** -8      # unit roundoff of BF16 (8 significant bits, round to nearest even)


def _abs_layers(wts, x, n, band):
    """Magnitude bounds of the three layers: A_l = |W_l| * A_(l-1) from
    A_0 = |x| (the convolutions of the absolute values, no ReLU), so that
    |z_l| <= A_l at every band vertex."""
    out, A = [], np.abs(x)
    for Wl in onet.split_params(np.abs(wts.astype(np.float64))):
        A = onet.conv(A, Wl, n, band)
        out.append(A)
    return out


def _band_edge(n, band):
    """Band vertices with a 27-neighbour off the band (where zero padding
    enters the stencil)."""
    off = np.zeros(band.size, dtype=bool)
    nb = band.astype(np.float64)[None]
    for tap in onet.TAPS:
        off |= onet.shift(nb, tap, n)[0] < 0.5
    return band.astype(bool) & off


def test_forward_elementwise_bound(setup):
    """Every output entry, band-edge vertices included, within the rounding
    bound of the BF16 path: each layer rounds its input and its weights to
    BF16 (relative u = 2^-8 each) and the hidden outputs once more, so with
    A_l the convolution of magnitudes the error of layer l is at most
    3u A_1, 6u A_2 and 8u A_3 for the output; checked with 9u A_3."""
    import torch
    w, P, D, band, lmu, net, wts = setup
    r = iss_inputs.random_vector(3, w["n"], seed=13)
    net.features(to_dev(r))
    y = torch.empty(net.band_size * 4, dtype=torch.float32, device="cuda")
    net.forward(y)
    x, su, sp, oy, _ = _oracle_forward(w, D, band, lmu, wts, r)
    A3 = _abs_layers(wts, x, w["n"], band)[2]
    bidx = np.nonzero(band)[0]
    got = to_host(y).reshape(-1, 4).T                  # (4, M) band order
    err = np.abs(got - oy[:, bidx])
    bound = 9.0 * U_BF16 * A3[:, bidx] + 1e-30
    worst = np.unravel_index(np.argmax(err / bound), err.shape)
    assert np.all(err <= bound), ("entry", worst, err[worst], bound[worst])
    edge = _band_edge(w["n"], band)[bidx]
    assert edge.any() and np.all(err[:, edge] <= bound[:, edge])


def test_backward_elementwise_bound(setup):
    """Every weight-gradient entry of the MSE loss within a rounding bound:
    G = the backward pass of magnitudes (|W|, the forward bounds A_l as
    activations, every ReLU open) driven by |dL/dy| plus the effect of the
    forward error on dL/dy (2/m of 8u A_3); the BF16 path rounds dL/dy,
    every back-propagated gradient, weights and activations (u each), so
    each entry is held to 16u G."""
    import torch
    w, P, D, band, lmu, net, wts = setup
    n = w["n"]
    r = iss_inputs.random_vector(3, n, seed=14)
    e = iss_inputs.random_vector(3, n, seed=15)
    net.features(to_dev(r))
    net.forward()
    t = torch.empty(net.band_size * 4, dtype=torch.float32, device="cuda")
    net.targets(to_dev(e), t)
    g = torch.empty(net.num_params, dtype=torch.float32, device="cuda")
    net.backward(t, g)
    x, su, sp, y, cache = _oracle_forward(w, D, band, lmu, wts, r)
    tgt = onet.scale_targets(3, n, e, band, su, sp, lmu, 1.0 / 12.0)
    _, dy = onet.mse(y, tgt, band)
    og = onet.backward(wts.astype(np.float64), cache, dy, n, band)
    A1, A2, A3 = _abs_layers(wts, x, n, band)
    m = band.sum() * 4
    dy_abs = (np.abs(dy) + 2.0 / m * 8.0 * U_BF16 * A3) * band
    G = onet.backward(np.abs(wts.astype(np.float64)), (np.abs(x), A1, A1, A2, A2), dy_abs, n, band)
    err = np.abs(to_host(g) - og)
    bound = 16.0 * U_BF16 * G + 1e-30
    k = int(np.argmax(err / bound))
    assert np.all(err <= bound), (k, err[k], bound[k], og[k])


def test_backward_parity(setup):
    import torch
    w, P, D, band, lmu, net, wts = setup
    r = iss_inputs.random_vector(3, w["n"], seed=9)
    e = iss_inputs.random_vector(3, w["n"], seed=10)
    net.features(to_dev(r))
    net.forward()
    t = torch.empty(net.band_size * 4, dtype=torch.float32, device="cuda")
    net.targets(to_dev(e), t)
    g = torch.empty(net.num_params, dtype=torch.float32, device="cuda")
    loss = net.backward(t, g)
    x, su, sp, y, cache = _oracle_forward(w, D, band, lmu, wts, r)
    tgt = onet.scale_targets(3, w["n"], e, band, su, sp, lmu, 1.0 / 12.0)
    assert np.allclose(to_host(t).reshape(-1, 4), tgt[:, band].T, rtol=1e-6, atol=1e-6)
    oloss, dy = onet.mse(y, tgt, band)
    og = onet.backward(wts.astype(np.float64), cache, dy, w["n"], band)
    assert abs(loss - oloss) <= 2e-2 * oloss
    gg = to_host(g)
    err = np.linalg.norm(gg - og) / np.linalg.norm(og)
    assert err < 3e-2, err
    # per layer too (no layer hidden by the others)
    o = 0
    for ci, co in onet.LAYERS:
        k = co * ci * 27
        el = np.linalg.norm(gg[o:o + k] - og[o:o + k]) / np.linalg.norm(og[o:o + k])
        assert el < 5e-2, (ci, co, el)
        o += k


def test_adam_parity():
    import torch
    from paper_1604_07994_amd.binding import adam_step
    rng = np.random.default_rng(11)
    w = rng.normal(size=1000)
    g = rng.normal(size=1000)
    m = np.zeros(1000)
    v = np.zeros(1000)
    wt = torch.tensor(w, dtype=torch.float32, device="cuda")
    mt = torch.zeros(1000, dtype=torch.float32, device="cuda")
    vt = torch.zeros_like(mt)
    gt = torch.tensor(g, dtype=torch.float32, device="cuda")
    for step in (1, 2, 3):
        adam_step(wt, mt, vt, gt, 1e-2, step)
        w, m, v = onet.adam(w, g, m, v, step, 1e-2)
    torch.cuda.synchronize()
    assert np.allclose(wt.cpu().numpy(), w, rtol=1e-5, atol=1e-6)


def test_safeguard_rejects_useless_or_broken_weights(setup):
    """A zero network changes nothing and a NaN network is rejected every
    time: the solve falls back to the plain V-cycle and still converges
    with the same iteration count."""
    import torch
    w, P, D, band, lmu, net, wts = setup
    b = torch.zeros(P.vector_size(), dtype=torch.float64, device="cuda")
    P.rhs_buoyancy(b, w["buoyant"])
    x = torch.zeros_like(b)
    plain = P.solve("interface", x, b, rtol=1e-8, maxit=200, raise_on_fail=False)
    net.attach(True)
    for fill in (0.0, float("nan")):
        net.set_weights(torch.full((net.num_params,), fill, dtype=torch.float32, device="cuda"))
        x = torch.zeros_like(b)
        info = P.solve("interface", x, b, rtol=1e-8, maxit=200, raise_on_fail=False)
        assert info["relres"] <= 1e-8
        assert info["net_accepted"] == 0 and info["net_rejected"] >= info["iterations"]
        assert info["iterations"] == plain["iterations"]
    net.attach(False)
    net.set_weights(torch.from_numpy(wts).cuda())


def test_residual_loss_gradient_chain(setup):
    """Training objective ||r' - K c(r')||^2 / ||r'||^2: GPU correction,
    residual and parameter gradient (through K and the Jacobi output units)
    against the FP64 oracle with the assembled K."""
    import torch
    w, P, D, band, lmu, net, wts = setup
    n = w["n"]
    N = (n + 1) ** 3
    beta = 1.0 / 12.0
    r = iss_inputs.random_vector(3, n, seed=12)
    rd = to_dev(r)
    net.features(rd)
    net.forward()
    c = torch.empty_like(rd)
    net.correction(c)
    q = torch.empty_like(rd)
    P.residual("interface", c, rd, q)
    nr = P.dot(rd, rd)
    kq = torch.empty_like(rd)
    P.apply("interface", q, kq)
    net.output_grad(kq, -2.0 / nr)
    g = torch.empty(net.num_params, dtype=torch.float32, device="cuda")
    net.backward(None, g)
    x, su, sp, y, cache = _oracle_forward(w, D, band, lmu, wts, r)
    free = D.free_mask()
    co = onet.correction(3, n, y, band, su, sp, lmu, beta) * free
    assert np.linalg.norm(to_host(c) - co) <= 2e-2 * np.linalg.norm(co)
    K = D.stokes("interface")
    qo = r - K @ co
    dldc = -2.0 * (K @ qo) / (r @ r)
    du, dp = onet.diagonal_scales(n, np.where(band, lmu, 0.0), beta)
    dy = np.zeros((4, N))
    dy[:3] = dldc[:3 * N].reshape(3, N) * su / du * free[:3 * N].reshape(3, N)
    dy[3] = dldc[3 * N:] * sp / dp
    dy *= band
    og = onet.backward(wts.astype(np.float64), cache, dy, n, band)
    gg = to_host(g)
    assert np.linalg.norm(gg - og) <= 3e-2 * np.linalg.norm(og)


def test_learned_gain_report(capsys):
    """What the trained network (weights/band_net.npz, trained on 10^4
    solver-generated pairs by paper_1604_07994_amd.learned) gains over the
    plain preconditioner on held-out geometries: FGMRES iterations and time
    to 1e-8, plain and with the correction attached, printed.  Both runs
    must converge; the gain itself is reported, not asserted (it may be
    zero or negative)."""
    import json
    import os
    from paper_1604_07994_amd import learned
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                        "paper_1604_07994_amd", "weights", "band_net.npz")
    wts = np.load(path, allow_pickle=False)["weights"]
    rows = learned.evaluate(wts, [100000, 100001], levels=6, log=lambda s: None)
    for r in rows:
        assert r["plain_relres"] <= 1e-8 and r["net_relres"] <= 1e-8, r
        assert r["net_accepted"] + r["net_rejected"] >= r["net_iterations"], r
    summary = learned.summarise(rows)
    with capsys.disabled():
        print("\nlearned band correction, held-out seeds 100000-100001: " + json.dumps(summary))
