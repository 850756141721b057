"""iss_smooth_noalloc, the allocation-free variant of iss_smooth: called
through the C ABI it gives the same bits as iss_smooth on the same input
(the same kernels on a static per-GPU scratch instead of per-level
buffers), on two calls in a row with the second on a smaller level (the
scratch keeps the first call's contents), in FP64 and FP32; a level larger
than the scratch is rejected with ISS_E_INVAL and leaves x untouched."""
import ctypes

import pytest

import iss_inputs
from tests.gpu_common import gpu_problem, small_workload, to_dev

pytestmark = pytest.mark.gpu


def _smooth_noalloc_raw(P, form, level, x, b, nsteps):
    from paper_1604_07994_amd import binding
    L = binding.lib()
    return L.iss_smooth_noalloc(P._h, binding.FORMS[form], level, binding._prec(x), nsteps,
                                ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(b.data_ptr()),
                                binding._stream())


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("form", ["strain", "interface"])
def test_noalloc_matches_smooth_on_two_calls(form, prec):
    import torch
    dt = torch.float64 if prec == "fp64" else torch.float32
    w = small_workload("sinker_3d", 4)          # levels 2..4: 33^3, then 17^3
    P = gpu_problem(w)
    for level, seed in ((4, 150), (3, 152)):
        n = w["macro"] * 2 ** level
        x = to_dev(iss_inputs.random_vector(3, n, seed=seed), dt)
        b = to_dev(iss_inputs.random_rhs(3, n, seed=seed + 1), dt)
        xa, xn = x.clone(), x.clone()
        P.smooth(form, xa, b, nsteps=2, level=level)
        assert _smooth_noalloc_raw(P, form, level, xn, b, 2) == 0
        torch.cuda.synchronize()
        assert torch.equal(xa, xn), (level, (xa - xn).abs().max().item())
        assert not torch.equal(xn, x)
    P.close()


def test_noalloc_rejects_levels_beyond_the_scratch():
    import torch
    w = small_workload("square_split_2d", 10)   # 1025^2: 3 x 3 x Ns doubles > 32 MiB
    P = gpu_problem(w)
    x = to_dev(iss_inputs.random_vector(2, w["n"], seed=154))
    b = to_dev(iss_inputs.random_rhs(2, w["n"], seed=155))
    x0 = x.clone()
    assert _smooth_noalloc_raw(P, "interface", w["levels"], x, b, 1) == -1
    from paper_1604_07994_amd import binding
    assert b"no-allocation scratch" in binding.lib().iss_last_error()
    torch.cuda.synchronize()
    assert torch.equal(x, x0)
    # the next level down fits and matches iss_smooth
    n = w["macro"] * 2 ** (w["levels"] - 1)
    x = to_dev(iss_inputs.random_vector(2, n, seed=156))
    b = to_dev(iss_inputs.random_rhs(2, n, seed=157))
    xa = x.clone()
    P.smooth("interface", xa, b, nsteps=1, level=w["levels"] - 1)
    assert _smooth_noalloc_raw(P, "interface", w["levels"] - 1, x, b, 1) == 0
    torch.cuda.synchronize()
    assert torch.equal(x, xa)
    P.close()
