"""Parity at the full workload sizes (65^3 sphere, 257^3 sinker) in the
configuration the benchmark times: operator applies on a seeded random
vector, compared with the oracle row by row on sampled vertices (random,
interface and boundary vertices), and vertex classification on the same
sample.  Tolerance as for the small cases: 1e-12 of the row's |K||x|."""
import numpy as np
import pytest

import iss_inputs
from oracle import assemble
from tests.gpu_common import gpu_problem, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", params=["sphere_3d", "sinker_3d"])
def full(request):
    import torch
    w = iss_inputs.workload(request.param)
    P = gpu_problem(w, coarse_mu="average", coarse_form="strain")
    x = iss_inputs.random_vector(3, w["n"], seed=41)
    cls, nif, nbd = P.vertex_class()
    rng = np.random.default_rng(42)
    iface = np.nonzero(cls & 1)[0]
    bnd = np.nonzero(cls & 2)[0]
    sample = np.unique(np.concatenate([
        iss_inputs.sample_vertices(3, w["n"], 300, 43),
        rng.choice(iface, min(300, iface.size), replace=False),
        rng.choice(bnd, 60, replace=False)]))
    yield w, P, x, cls, sample
    P.close()
    torch.cuda.empty_cache()


def test_classification_sample(full):
    w, P, x, cls, sample = full
    D = assemble.sampled_rows(3, w["n"], w["inclusions"], w["mu"], sample)
    assert np.array_equal((cls[sample] & 1).astype(bool), D.interface[sample])
    assert np.array_equal((cls[sample] & 2).astype(bool), D.boundary[sample])


@pytest.mark.parametrize("form", ["interface", "strain", "gradient"])
def test_apply_sampled_rows(full, form):
    import torch
    w, P, x, cls, sample = full
    xg = to_dev(x)
    y = torch.empty_like(xg)
    P.apply(form, xg, y)
    yh = to_host(y)
    del xg, y
    N = (w["n"] + 1) ** 3
    verts, Y = assemble.sampled_stokes_rows(3, w["n"], w["inclusions"], w["mu"], sample, form, x)
    # |K||x| scale of the sampled rows
    _, S = assemble.sampled_stokes_rows(3, w["n"], w["inclusions"], w["mu"], sample, form, np.abs(x))
    scale = np.abs(S).max()
    got = np.stack([yh[f * N + verts] for f in range(4)])
    err = np.abs(got - Y).max()
    assert err <= 1e-12 * scale, (form, err, scale)
