"""GPU parity of the operator applies, residuals and right-hand side against
the CPU oracle's explicitly assembled matrices.

Tolerance (FP64): |y_gpu - y_oracle| <= 1e-12 * max_i (|K| |x|)_i, i.e.
relative to the largest row magnitude of the product (guards against
cancellation).  FP32: 2e-6 on the same scale (float epsilon times the
stencil length)."""
import numpy as np
import pytest

import iss_inputs
from oracle import problem as oprob
from tests.gpu_common import (abs_scale, assert_close_scaled, gpu_problem, oracle_disc,
                              small_workload, to_dev, to_host)

pytestmark = pytest.mark.gpu

CASES = [
    ("square_split_2d", 4, None),     # 17^2
    ("square_split_2d", 3, 3),        # 25^2, ragged rows
    ("square_split_2d", 6, None),     # 65^2 (full 2D workload)
    ("sphere_3d", 4, None),           # 17^3
    ("sphere_3d", 3, 3),              # 25^3 ragged
    ("sinker_3d", 3, None),           # 2 x 2 x 2 macro cubes, 17^3, 8 spheres
    ("sinker_3d", 3, 5),              # 41^3, several tiles + ragged tail
]


def _ids(c):
    return "%s-L%d-m%s" % c


@pytest.fixture(scope="module", params=CASES, ids=[_ids(c) for c in CASES])
def case(request):
    name, levels, macro = request.param
    w = small_workload(name, levels, macro)
    P = gpu_problem(w)
    D = oracle_disc(w)
    yield w, P, D
    P.close()


def test_vertex_classification(case):
    w, P, D = case
    cls, nif, nbd = P.vertex_class()
    assert np.array_equal((cls & 1).astype(bool), D.interface)
    assert np.array_equal((cls & 2).astype(bool), D.boundary)
    assert nif == int(D.interface.sum()) and nbd == int(D.boundary.sum())
    assert nif > 0


@pytest.mark.parametrize("form", ["gradient", "strain", "interface"])
@pytest.mark.parametrize("block", ["full", "velocity"])
def test_apply_fp64(case, form, block):
    import torch
    w, P, D = case
    x = iss_inputs.random_vector(w["dim"], w["n"], seed=11)
    if block == "full":
        K = D.stokes(form)
    else:
        import scipy.sparse as sp
        A = D.velocity_operator(form)
        K = sp.block_diag([A, sp.csr_matrix((D.N, D.N))]).tocsr()
    ref = K @ x
    y = torch.empty_like(to_dev(x))
    P.apply(form, to_dev(x), y, block=block)
    assert_close_scaled(to_host(y), ref, abs_scale(K, x), 1e-12, "%s/%s" % (form, block))


@pytest.mark.parametrize("form", ["strain", "interface"])
def test_apply_fp32(case, form):
    import torch
    w, P, D = case
    x = iss_inputs.random_vector(w["dim"], w["n"], seed=12)
    K = D.stokes(form)
    x32 = x.astype(np.float32).astype(np.float64)
    ref = K @ x32
    y = torch.empty(x.size, dtype=torch.float32, device="cuda")
    P.apply(form, to_dev(x, torch.float32), y)
    assert_close_scaled(to_host(y), ref, abs_scale(K, x32), 2e-6, form)


@pytest.mark.parametrize("form", ["strain", "interface"])
def test_apply_bf16_storage(case, form):
    """BF16-stored vectors, FP32 arithmetic: the input is the BF16 rounding
    of x, the output is rounded to BF16 once (unit roundoff 2^-8)."""
    import torch
    w, P, D = case
    x = iss_inputs.random_vector(w["dim"], w["n"], seed=13)
    xb = to_dev(x, torch.bfloat16)
    K = D.stokes(form)
    xr = to_host(xb)
    ref = K @ xr
    y = torch.empty(x.size, dtype=torch.bfloat16, device="cuda")
    P.apply(form, xb, y)
    err = np.abs(to_host(y) - ref)
    bound = 2.0 ** -8 * np.abs(ref) + 4e-6 * np.max(abs_scale(K, xr))
    assert np.all(err <= bound), (form, float(np.max(err - bound)))


@pytest.mark.parametrize("form", ["strain", "interface"])
def test_apply_fp16_storage(case, form):
    """FP16-stored vectors, FP32 arithmetic: the input is the FP16 rounding
    of x, the output is rounded to FP16 once (unit roundoff 2^-11; entries
    below 2^-14 are subnormal with spacing 2^-24)."""
    import torch
    w, P, D = case
    x = iss_inputs.random_vector(w["dim"], w["n"], seed=15)
    xh = to_dev(x, torch.float16)
    K = D.stokes(form)
    xr = to_host(xh)
    ref = K @ xr
    y = torch.empty(x.size, dtype=torch.float16, device="cuda")
    P.apply(form, xh, y)
    err = np.abs(to_host(y) - ref)
    bound = 2.0 ** -11 * np.abs(ref) + 4e-6 * np.max(abs_scale(K, xr)) + 2.0 ** -24
    assert np.all(err <= bound), (form, float(np.max(err - bound)))


@pytest.mark.parametrize("form", ["gradient", "strain", "interface"])
def test_residual_and_norms(case, form):
    import torch
    w, P, D = case
    x = iss_inputs.random_vector(w["dim"], w["n"], seed=13)
    b = iss_inputs.random_rhs(w["dim"], w["n"], seed=14)
    K = D.stokes(form)
    ref = b - K @ x
    r = torch.empty_like(to_dev(x))
    norms = P.residual(form, to_dev(x), to_dev(b), r, norms=True)
    rr = to_host(r)
    assert_close_scaled(rr, ref, abs_scale(K, x) + np.abs(b), 1e-12, form)
    N = D.N
    for f in range(w["dim"] + 1):
        assert np.isclose(norms[f], np.linalg.norm(ref[f * N:(f + 1) * N]), rtol=1e-10)
    assert np.isclose(norms[-1], np.linalg.norm(ref), rtol=1e-10)


def test_buoyancy_rhs(case):
    import torch
    w, P, D = case
    b = torch.zeros(P.vector_size(), dtype=torch.float64, device="cuda")
    P.rhs_buoyancy(b, w["buoyant"] or [1])
    ref = oprob.rhs_buoyancy(w["dim"], w["n"], D.elems, D.phase_e, w["buoyant"] or [1])
    ref = ref * D.free_mask()
    assert np.allclose(to_host(b), ref, rtol=1e-13, atol=1e-18)
