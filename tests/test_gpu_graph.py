"""The part of the V-cycle below the finest level is replayed from a HIP
graph after its first (eager) run.  Replays must give the same bits as
eager launches: several cycles in a row, with unrelated eager GPU work and
synchronisations between them, in FP64 and FP32, and through a whole FGMRES
solve.  ISS_VCYCLE_GRAPH=0 at problem creation selects eager launches."""
import os

import numpy as np
import pytest

import iss_inputs
from tests.gpu_common import gpu_problem, small_workload, to_dev

pytestmark = pytest.mark.gpu


def _problem(w, graphs, **kw):
    old = os.environ.get("ISS_VCYCLE_GRAPH")
    os.environ["ISS_VCYCLE_GRAPH"] = "1" if graphs else "0"
    try:
        return gpu_problem(w, **kw)
    finally:
        if old is None:
            del os.environ["ISS_VCYCLE_GRAPH"]
        else:
            os.environ["ISS_VCYCLE_GRAPH"] = old


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_graph_vcycle_matches_eager(prec):
    import torch
    dt = torch.float64 if prec == "fp64" else torch.float32
    # 32^3 sinkers, coarse level 8^3: the recorded part holds the 16^3
    # level (merged launches) and the dense coarse solve
    w = small_workload("sinker_3d", 4)
    Pe, Pg = _problem(w, False), _problem(w, True)
    for it in range(5):
        b = to_dev(iss_inputs.random_rhs(3, w["n"], seed=60 + it), dt)
        xe = torch.zeros_like(b)
        xg = torch.zeros_like(b)
        Pe.vcycle("strain", xe, b)
        Pg.vcycle("strain", xg, b)
        # unrelated eager work and a synchronisation between replays
        junk = torch.randn(1 << 20, device="cuda", dtype=torch.float64)
        assert torch.isfinite(junk.sum())
        torch.cuda.synchronize()
        assert torch.equal(xe, xg), (prec, it, (xe - xg).abs().max().item())
        assert torch.count_nonzero(xg).item() > 0
    Pe.close()
    Pg.close()


def test_graph_solve_matches_eager():
    """FGMRES with the default configuration of the benchmark (strain form
    below the finest level, averaged coarse viscosity): identical history
    and solution with and without the recorded coarse cycle."""
    import torch
    w = small_workload("sinker_3d", 4)
    kw = dict(outer="fgmres", coarse_mu="average", coarse_form="strain", mid_form="strain", nu_inc=2,
              omega=0.6)
    b = to_dev(iss_inputs.random_rhs(3, w["n"], seed=70))
    out = []
    for graphs in (False, True):
        P = _problem(w, graphs, **kw)
        x = torch.zeros_like(b)
        info = P.solve("interface", x, b, rtol=1e-8, maxit=120, raise_on_fail=False)
        out.append((x, np.array(info["history"]), info["status"]))
        P.close()
    (xe, he, se), (xg, hg, sg) = out
    assert se == sg
    assert np.array_equal(he, hg), np.abs(he - hg).max()
    assert torch.equal(xe, xg)
