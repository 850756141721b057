"""Shared helpers of the GPU parity tests: build matching HIP and oracle
problems from one workload description."""
import numpy as np

import iss_inputs
from oracle import assemble, mesh, multigrid as mg


def torch_dev():
    import torch
    return torch.device("cuda:0")


def to_dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(torch_dev())


def to_host(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().double().cpu().numpy()


def small_workload(name, levels, macro=None, seed=0):
    w = iss_inputs.workload(name, seed=seed, levels=levels)
    if macro is not None:
        w["macro"] = macro
        w["n"] = macro * 2 ** w["levels"]
    w["coarse"] = min(w["coarse"], w["levels"])
    return w


def gpu_problem(w, **kw):
    """Library problem for a workload; coarse levels use the centroid rule
    (the oracle hierarchy's rediscretisation) unless stated."""
    from paper_1604_07994_amd import Problem
    kw.setdefault("coarse_mu", "centroid")
    return Problem.from_workload(w, **kw)


def oracle_disc(w, level=None):
    n = w["n"] if level is None else w["macro"] * 2 ** level
    return assemble.Discretisation(w["dim"], n, w["inclusions"], w["mu"])


def abs_scale(K, x):
    """|K| |x| row-wise: the rounding scale of K x."""
    Ka = abs(K)
    return Ka @ np.abs(x)


def assert_close_scaled(y, ref, scale, tol, what=""):
    err = np.abs(y - ref)
    bound = tol * max(np.max(scale), 1e-300)
    worst = int(np.argmax(err))
    assert err.max() <= bound, "%s: max err %.3e > %.3e at %d (y=%.6e ref=%.6e)" % (
        what, err.max(), bound, worst, y[worst], ref[worst])
