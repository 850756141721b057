"""Benchmark: seconds to a 1e-8 relative residual and stencil GB/s, decoupled
(interface) vs strain form, on one MI355X.

Workload (default): sinker_3d -- unit cube as 2 x 2 x 2 macro cubes (48 Kuhn
tetrahedra) refined 7 times (257^3 vertices, 6.79e7 unknowns u, v, w, p),
8 seeded spheres (seed 0) with viscosity 1e4 inside and 1 outside, buoyancy
rho = 1 inside, no-slip walls.  Synthetic, seeded, generated on the device by
the library (iss_rhs_buoyancy).  One "step" is one complete solve from x = 0
to ||b - K x|| <= 1e-8 ||b|| with the interface (decoupled + a_tr interface
rows) form in FP64: FGMRES(150) preconditioned by two stationary Uzawa
V_var(4,4) cycles (two more smoothing steps per coarser level, omega 0.8,
element-averaged coarse viscosity, strain form on every level below the
finest); the strain form is timed with the same solver.  The paper's own
configuration (a_tr on every level but the coarsest) is run once for the
record.

Prints one JSON line.  --gpus N with N > 1 exits: the library runs on one GPU.
"""
import argparse
import hashlib
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="sinker_3d")
    ap.add_argument("--levels", type=int, default=None)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--omega", type=float, default=0.8)
    ap.add_argument("--nu", type=int, default=4, help="pre- and post-smoothing steps")
    ap.add_argument("--nu-inc", type=int, default=2,
                    help="variable V-cycle: extra smoothing steps per level below the finest")
    ap.add_argument("--cycles", type=int, default=2, help="stationary V-cycles per preconditioner application")
    ap.add_argument("--mid-form", default="strain", choices=["same", "strain", "interface", "gradient"],
                    help="viscous form of the levels between the finest and the coarsest")
    ap.add_argument("--rate-iters", type=int, default=200,
                    help="cycles of the asymptotic-rate measurement (0: skip)")
    ap.add_argument("--no-paper-config", action="store_true",
                    help="skip the run with a_tr on every level but the coarsest")
    ap.add_argument("--restart", type=int, default=150)
    ap.add_argument("--maxit", type=int, default=400)
    ap.add_argument("--outer", default="fgmres")
    ap.add_argument("--coarse-mu", default="average", choices=["average", "centroid"])
    ap.add_argument("--forms", default="interface,strain")
    ap.add_argument("--coarse-form", default="strain", choices=["same", "strain", "interface", "gradient"],
                    help="viscous form of the coarsest level (the swap of Sec. 5)")
    ap.add_argument("--kernels-only", action="store_true",
                    help="no solves: smoothing steps, applies and a plain copy (for profiler runs)")
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the learned band-correction comparison (65^3 held-out geometries)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--quick", action="store_true", help="solves only, no apply/smoother timing")
    ap.add_argument("--cpu-full", action="store_true",
                    help="also time complete oracle solves of the 65^2 and 65^3 workloads (minutes of CPU)")
    ap.add_argument("--no-columns", action="store_true",
                    help="skip the viscosity-columns timing problem of the paper (257^3, free-slip)")
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def event_time(fn, reps):
    """Average milliseconds of fn() over reps calls, HIP events on torch's
    current stream (the stream the library launches on)."""
    import torch
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    fn()
    torch.cuda.synchronize()
    s.record()
    for _ in range(reps):
        fn()
    e.record()
    torch.cuda.synchronize()
    return s.elapsed_time(e) / reps


def cpu_baseline(w, its_gpu, omega, nu, restart, nu_inc, cycles, mid_form, coarse_form, sample_its=8):
    """The oracle (explicit CSR, same algorithm and settings) on one host
    core: FGMRES iterations of the same workload family at 65^3 (the 257^3
    CSR would need ~40 GB), timed, and scaled to the full lattice by vertex
    count and to the GPU's iteration count."""
    code = r"""
import json, sys, time, numpy as np
sys.path.insert(0, %r)
import iss_inputs
from oracle import multigrid as mg, problem as oprob
w = iss_inputs.workload(%r, seed=%d, levels=%d)
H = mg.Hierarchy(w['dim'], w['macro'], w['levels'], w['coarse'], w['inclusions'], w['mu'], 'interface',
                 omega=%r, nu1=%d, nu2=%d, coarse_mu='average', coarse_form=%r, mid_form=%r, nu_inc=%d)
lv = H.levels[w['levels']]
b = oprob.rhs_buoyancy(w['dim'], w['n'], lv.disc.elems, lv.disc.phase_e, w['buoyant']) * lv.free
t = time.time()
x, h = mg.solve_fgmres(H, b, rtol=1e-8, restart=%d, maxit=%d, cycles=%d)
dt = time.time() - t
print(json.dumps({'seconds': dt, 'its': len(h) - 1, 'N': lv.N, 'relres': float(h[-1])}))
"""
    lv_small = min(w["levels"], 5)
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    src = code % (ROOT, w["name"], w.get("seed", 0), lv_small, omega, nu, nu, coarse_form, mid_form, nu_inc,
                  restart, sample_its, cycles)
    out = subprocess.run([sys.executable, "-c", src], capture_output=True, text=True, env=env, timeout=900)
    if out.returncode != 0:
        raise RuntimeError(out.stderr[-2000:])
    r = json.loads(out.stdout.strip().splitlines()[-1])
    per_it_vertex = r["seconds"] / max(r["its"], 1) / r["N"]
    N_full = (w["n"] + 1) ** w["dim"]
    est = per_it_vertex * N_full * its_gpu
    return {"value": est, "unit": "s", "cores": 1, "host_nproc": os.cpu_count(), "kind": "oracle",
            "sample": "oracle FGMRES with the same preconditioner (%d stationary V-cycles, same smoothing and "
                      "coarse settings) on %s refined %d times (%d vertices): %d iterations in %.1f s on one "
                      "core, scaled by vertex count to %d vertices and to the GPU's %d iterations"
                      % (cycles, w["name"], lv_small, r["N"], r["its"], r["seconds"], N_full, its_gpu)}


ORACLE_SOLVE = r"""
import json, sys, time, numpy as np
sys.path.insert(0, %r)
import iss_inputs
from oracle import multigrid as mg, problem as oprob
w = iss_inputs.workload(%r)
H = mg.Hierarchy(w['dim'], w['macro'], w['levels'], w['coarse'], w['inclusions'], w['mu'], %r,
                 omega=%r, nu1=%d, nu2=%d, coarse_mu='average', coarse_form=%r, mid_form=%r, nu_inc=%d)
lv = H.levels[w['levels']]
if w['buoyant']:
    b = oprob.rhs_buoyancy(w['dim'], w['n'], lv.disc.elems, lv.disc.phase_e, w['buoyant']) * lv.free
else:
    b = iss_inputs.random_rhs(w['dim'], w['n'], seed=%d)
t = time.time()
x, h = mg.solve_fgmres(H, b, rtol=1e-8, restart=%d, maxit=%d, cycles=%d)
dt = time.time() - t
print(json.dumps({'seconds': dt, 'its': len(h) - 1, 'relres': float(h[-1])}))
"""


def _gpu_full_solves(Problem, name, cfg, args, forms, rhs_seed):
    """GPU leg of full_solves: median of 3 timed solves after one warm-up."""
    import torch
    import iss_inputs
    w = iss_inputs.workload(name)
    P = Problem.from_workload(w, outer="fgmres", restart=args.restart, coarse_mu="average", nu1=cfg["nu"],
                              nu2=cfg["nu"], nu_inc=cfg["nu_inc"], omega=cfg["omega"],
                              coarse_form=cfg["coarse_form"], mid_form=cfg["mid_form"], cycles=cfg["cycles"])
    try:
        if w["buoyant"]:
            b = torch.zeros(P.vector_size(), dtype=torch.float64, device="cuda")
            P.rhs_buoyancy(b, w["buoyant"])
        else:
            b = torch.from_numpy(iss_inputs.random_rhs(w["dim"], w["n"], seed=rhs_seed)).cuda()
        res = {}
        for form in forms:
            x = torch.zeros_like(b)
            times = []
            for rep in range(4):
                x.zero_()
                torch.cuda.synchronize()
                t = time.perf_counter()
                info = P.solve(form, x, b, rtol=1e-8, maxit=args.maxit, raise_on_fail=False)
                torch.cuda.synchronize()
                if rep > 0:
                    times.append(time.perf_counter() - t)
            res[form] = {"gpu_seconds": sorted(times)[1], "gpu_iterations": info["iterations"],
                         "gpu_relres": info["relres"]}
        return res
    finally:
        P.close()


def full_solves(Problem, args, mid_form, coarse_form, forms, rhs_seed=177):
    """Complete solves to 1e-8 of the two small workloads, measured on both
    sides, nothing scaled: the GPU (median of 3 after one warm-up) and the
    oracle on one host core per form (one run; setup and assembly
    excluded).  The 65^2 split square (mu 10 / 1, seeded U[-1, 1] forcing)
    with the plain multigrid of Sec. 5 (FGMRES(150) around one V(3,3)
    cycle, omega 0.3, each form on every level); the 65^3 sphere (mu 1e3,
    buoyancy) with the benchmark's solver."""
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    bench_cfg = dict(omega=args.omega, nu=args.nu, nu_inc=args.nu_inc, cycles=args.cycles, mid_form=mid_form,
                     coarse_form=coarse_form)
    plain_cfg = dict(omega=0.3, nu=3, nu_inc=0, cycles=1, mid_form=None, coarse_form=None)
    out = {}
    for name, label, cfg in (("square_split_2d", "square_split_2d 65^2 mu 10/1", plain_cfg),
                             ("sphere_3d", "sphere_3d 65^3 mu 1e3", bench_cfg)):
        procs = {}
        for form in forms:          # the oracle runs in the background while the GPU solves
            src = ORACLE_SOLVE % (ROOT, name, form, cfg["omega"], cfg["nu"], cfg["nu"], cfg["coarse_form"],
                                  cfg["mid_form"], cfg["nu_inc"], rhs_seed, args.restart, args.maxit,
                                  cfg["cycles"])
            procs[form] = subprocess.Popen([sys.executable, "-c", src], stdout=subprocess.PIPE,
                                           stderr=subprocess.PIPE, text=True, env=env)
        try:
            res = _gpu_full_solves(Problem, name, cfg, args, forms, rhs_seed)
        except BaseException:
            for pr in procs.values():       # no oracle run outlives a failed GPU leg
                pr.kill()
                pr.wait()
            raise
        for form, pr in procs.items():
            so, se = pr.communicate(timeout=900)
            if pr.returncode != 0:
                raise RuntimeError(se[-2000:])
            r = json.loads(so.strip().splitlines()[-1])
            res[form].update({"oracle_seconds": r["seconds"], "oracle_iterations": r["its"],
                              "oracle_relres": r["relres"],
                              "oracle_over_gpu": r["seconds"] / res[form]["gpu_seconds"]})
        out[label] = {"solver": "fgmres(%d), %d V(%d,%d) cycle(s) +%d per coarser level, omega %.2f, levels "
                                "below the finest: %s, coarsest: %s" % (args.restart, cfg["cycles"], cfg["nu"],
                                                                      cfg["nu"], cfg["nu_inc"], cfg["omega"],
                                                                      cfg["mid_form"] or "same form",
                                                                      cfg["coarse_form"] or "same form"),
                      "forms": res}
        log("full solves %s: %s" % (label, {f: (v["gpu_iterations"], v["oracle_iterations"],
                                                 round(v["gpu_seconds"], 4), round(v["oracle_seconds"], 2))
                                             for f, v in res.items()}))
    return out


def measured_traffic(kernel, form):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 PMC
    summary (FETCH_SIZE and WRITE_SIZE, each scaled by the same counter's
    reading for a plain copy of known size), or None when the kernel source
    or the host layout code has changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    entry = rec.get("%s/%s" % (kernel, form))
    if not entry or rec.get("sources_sha256") != kernel_sources_digest():
        return None
    return entry["bytes_per_launch"]


def kernel_sources_digest():
    """SHA-256 over the kernel source and the host source that fixes the
    data layout the kernels stream (the counters are valid for both)."""
    h = hashlib.sha256()
    for name in ("iss_kernels.hip", "iss_host.cpp"):
        with open(os.path.join(ROOT, "paper_1604_07994_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


# Sec. 5, Table timeANDconv: time of one V_var(3,3) cycle and asymptotic
# rate per form on the viscosity-columns problem, level 6 (257^3), on a
# 32-core Xeon server: for comparison only (another machine)
PAPER_COLUMNS_L6 = {"strain": {"cycle_s": 3.02, "rate": 0.280},
                    "interface": {"cycle_s": 2.45, "rate": 0.242},
                    "gradient": {"cycle_s": 2.64, "rate": 0.240}}


def columns_report(rate_iters, reps=5):
    """The paper's timing problem: viscosity columns (mu 1 / 10, free-slip)
    at 257^3 with its multigrid settings (Uzawa V(3,3) with 2 more steps per
    coarser level, omega 0.3, averaged coarse viscosity, its coarse grid at
    level 2 solved by preconditioned MINRES, for a_tr in the strain form with
    the momentum right-hand side modified by B^T M^-1 r_2):
    per form the time of one V-cycle (HIP events), the asymptotic rate and
    the stationary iterations to 1e-8 from zero; then cycle time and rate
    with the hierarchy continued to a 9^3 direct coarse solve."""
    import numpy as np
    import torch
    import iss_inputs
    from paper_1604_07994_amd import Problem
    w = iss_inputs.workload("columns_3d")
    # the paper's coarse grid: level 2 (17^3, 19 652 unknowns), MINRES there;
    # a_tr is swapped for the strain form there (with the modified right-hand
    # side), the strain and gradient forms keep their own
    wp = dict(w, coarse=2)
    base = dict(outer="richardson", omega=0.3, nu1=3, nu2=3, nu_inc=2, coarse_mu="average")
    dev = torch.device("cuda:0")
    fn = torch.from_numpy(np.ascontiguousarray(iss_inputs.column_force(3, w["n"]).ravel())).to(dev)
    x0 = torch.from_numpy(iss_inputs.random_vector(3, w["n"], seed=8, bc="freeslip")).to(dev)
    out, sol = {}, {}
    P = None
    for form in ("interface", "strain", "gradient"):
        if P is not None:
            P.close()
        swap = dict(coarse_form="strain", coarse_rhs_mod=True) if form == "interface" else {}
        P = Problem.from_workload(wp, coarse_solver="minres", minres_iters=30, minres_cg=5, **base, **swap)
        b = torch.empty(P.vector_size(), dtype=torch.float64, device=dev)
        P.rhs_nodal_force(fn, b)
        x = torch.zeros_like(b)
        P.vcycle(form, x, b)
        ms = event_time(lambda: P.vcycle(form, x, b), reps)
        hist = P.asymptotic_rate(form, x0.clone(), iters=rate_iters) if rate_iters > 0 else [float("nan")]
        x.zero_()
        info = P.solve(form, x, b, rtol=1e-8, maxit=60, raise_on_fail=False)
        out[form] = {"cycle_ms": ms, "rate": hist[-1], "rate_iterations": rate_iters,
                     "iterations_to_1e-8": info["iterations"], "relres": info["relres"],
                     "solve_s": info["seconds"], "paper_xeon32": PAPER_COLUMNS_L6[form]}
        log("columns %s: V-cycle %.2f ms, rate %.4f, %d its to %.1e in %.3f s" %
            (form, ms, hist[-1], info["iterations"], info["relres"], info["seconds"]))
        # on to 1e-11 for the comparison of the discrete solutions below
        P.solve(form, x, b, rtol=1e-11, maxit=60, raise_on_fail=False)
        sol[form] = x
    # Sec. 4 columns tables (P1-P1, level 6): relative differences to the
    # strain-form solution in the velocity L2 norm and in ||v||_V^2 = a_sym(v, v)
    N = P.num_vertices()
    m, y = torch.empty_like(b), torch.empty_like(b)

    def norms(e):
        P.rhs_nodal_force(e[:3 * N].contiguous(), m)
        P.apply("strain", e, y, block="velocity")
        return (float(torch.dot(e[:3 * N], m[:3 * N])) ** 0.5, float(torch.dot(e[:3 * N], y[:3 * N])) ** 0.5)

    ref = norms(sol["strain"])
    paper_tab = {"interface": (7.5985e-05, 1.6675e-03), "gradient": (2.0098e-02, 4.2121e-02)}
    diffs = {}
    for form in ("interface", "gradient"):
        d = norms(sol[form] - sol["strain"])
        diffs[form + "_vs_strain"] = {"l2": d[0] / ref[0], "V": d[1] / ref[1],
                                      "paper_l2": paper_tab[form][0], "paper_V": paper_tab[form][1]}
    log("columns differences to the strain solution: %s" % diffs)
    P.close()
    # the same multigrid continued to a 9^3 level solved directly
    direct = {}
    for form in ("interface", "strain", "gradient"):
        swap = dict(coarse_form="strain", coarse_rhs_mod=True) if form == "interface" else {}
        Pd = Problem.from_workload(w, **base, **swap)
        x = torch.zeros_like(b)
        Pd.vcycle(form, x, b)
        ms = event_time(lambda: Pd.vcycle(form, x, b), reps)
        hist = Pd.asymptotic_rate(form, x0.clone(), iters=rate_iters) if rate_iters > 0 else [float("nan")]
        direct[form] = {"cycle_ms": ms, "rate": hist[-1]}
        Pd.close()
    log("columns, 9^3 direct coarse solve: %s" % direct)
    return {"workload": "columns_3d: 257^3 vertices, mu 1 / 10 columns (0,1/4)^2 x (0,1) and (3/4,1)^2 x (0,1), "
                        "free-slip, f = (0, 0, -cos 2 pi x cos 2 pi y sin pi z)",
            "cycle": "Uzawa V(3,3) +2 steps per coarser level, omega 0.3, averaged coarse viscosity, FP64; "
                     "coarsest level 17^3 (the paper's level 2) solved by 30 MINRES steps preconditioned with 5 "
                     "Jacobi-CG steps and the lumped pressure mass, in the strain form with the modified "
                     "momentum right-hand side for the interface form, in their own form for the others",
            "direct_coarse_9": direct,
            "forms": out,
            "strain_over_interface_cycle": out["strain"]["cycle_ms"] / out["interface"]["cycle_ms"],
            "solution_differences_level6": diffs}


def learned_report(seeds=(100000, 100004)):
    """Plain vs learned-corrected FGMRES on held-out 65^3 inclusion
    geometries with the stored trained weights (weights/band_net.npz)."""
    import numpy as np
    from paper_1604_07994_amd import learned
    path = os.path.join(ROOT, "paper_1604_07994_amd", "weights", "band_net.npz")
    w = np.load(path, allow_pickle=False)["weights"]
    rows = learned.evaluate(w, list(seeds), levels=6, log=log)
    return {"workload": "learned_3d 65^3, held-out seeds %s" % (list(seeds),),
            "plain_iterations": [r["plain_iterations"] for r in rows],
            "net_iterations": [r["net_iterations"] for r in rows],
            "plain_seconds": [r["plain_seconds"] for r in rows],
            "net_seconds": [r["net_seconds"] for r in rows],
            "net_accepted": [r["net_accepted"] for r in rows],
            "net_rejected": [r["net_rejected"] for r in rows]}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: the library runs on one GPU only; --gpus %d is not supported" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    import torch
    import iss_inputs
    from paper_1604_07994_amd import Problem

    w = iss_inputs.workload(args.workload, seed=args.seed, levels=args.levels)
    w["seed"] = args.seed
    dev = torch.device("cuda:0")
    forms = args.forms.split(",")
    t0 = time.time()
    mid_form = None if args.mid_form == "same" else args.mid_form
    coarse_form = None if args.coarse_form == "same" else args.coarse_form
    P = Problem.from_workload(w, outer=args.outer, omega=args.omega, restart=args.restart,
                              coarse_mu=args.coarse_mu, nu1=args.nu, nu2=args.nu, nu_inc=args.nu_inc,
                              coarse_form=coarse_form, mid_form=mid_form, cycles=args.cycles)
    log("setup %.1f s, n = %d" % (time.time() - t0, w["n"]))
    nvec = P.vector_size()
    N = P.num_vertices()
    cls, nif, nbd = P.vertex_class()
    b = torch.zeros(nvec, dtype=torch.float64, device=dev)
    P.rhs_buoyancy(b, w["buoyant"] or [1])
    x = torch.zeros_like(b)

    if args.kernels_only:
        # fixed, small launch sequence for profiler runs: one smoothing step
        # per form, the stencil applies, and a plain device copy of known
        # size (scales the HBM byte counters)
        xr = torch.rand(nvec, dtype=torch.float64, device=dev)
        y = torch.empty_like(xr)
        for _ in range(args.reps):
            for form in forms:
                P.smooth(form, x, b, 1)
            for form in forms:
                P.apply(form, xr, y, block="velocity")
                P.apply(form, xr, y, block="full")
            torch.mul(xr, 1.0, out=y)        # plain read + write of one vector
        torch.cuda.synchronize()
        log("kernels-only: %d reps, elementwise copy of %d bytes read + written per rep"
            % (args.reps, xr.numel() * 8))
        return

    results = {}
    for form in forms:
        for _ in range(args.warmup):
            x.zero_()
            info = P.solve(form, x, b, rtol=1e-8, maxit=args.maxit, raise_on_fail=False)
            log("warmup %s: its %d relres %.2e %.3f s" % (form, info["iterations"], info["relres"], info["seconds"]))
        steps = args.steps if form == forms[0] else max(1, min(args.steps, 2))
        times = []
        for _ in range(steps):
            x.zero_()
            torch.cuda.synchronize()
            t = time.perf_counter()
            info = P.solve(form, x, b, rtol=1e-8, maxit=args.maxit, raise_on_fail=False)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t)
            log("%s: its %d relres %.2e %.3f s" % (form, info["iterations"], info["relres"], times[-1]))
        results[form] = {"seconds": sorted(times)[len(times) // 2], "all": times,
                         "iterations": info["iterations"], "relres": info["relres"],
                         "status": info["status"]}
        if form == forms[0]:
            x64 = x.clone()                  # FP64 solution of the main form
    def field_errors(xm):
        """relative L2 difference per field to the FP64 solve (pressure means
        removed: the constant pressure is the null space of K)"""
        out = []
        for f in range(w["dim"] + 1):
            a, c = xm[f * N:(f + 1) * N], x64[f * N:(f + 1) * N]
            if f == w["dim"]:
                a, c = a - a.mean(), c - c.mean()
            out.append(float(torch.linalg.norm(a - c) / torch.linalg.norm(c)))
        return out

    fp32 = storage16 = None
    if not args.no_fp32:
        # FP32 V-cycle inside the FP64 FGMRES: the mixed-precision result
        fp32 = {}
        x.zero_()
        P.solve(forms[0], x, b, prec="fp32", rtol=1e-8, maxit=args.maxit, raise_on_fail=False)
        x.zero_()
        torch.cuda.synchronize()
        t = time.perf_counter()
        info = P.solve(forms[0], x, b, prec="fp32", rtol=1e-8, maxit=args.maxit, raise_on_fail=False)
        torch.cuda.synchronize()
        fp32["fp32"] = {"seconds": time.perf_counter() - t, "iterations": info["iterations"],
                        "relres": info["relres"], "status": info["status"],
                        "rel_error_per_field_vs_fp64": field_errors(x)}
        fp32["fp32"]["speedup_vs_fp64"] = results[forms[0]]["seconds"] / fp32["fp32"]["seconds"]
        log("fp32-preconditioned %s: its %d relres %.2e %.3f s" % (forms[0], info["iterations"], info["relres"],
                                                                 fp32["fp32"]["seconds"]))
        # 16-bit storage (FP32 arithmetic): on this workload, capped at 100
        # iterations (they stall at contrast 1e4), and on the 65^3 sphere
        # (contrast 1e3), where they converge
        storage16 = {}
        for prec in ("bf16", "fp16"):
            x.zero_()
            info = P.solve(forms[0], x, b, prec=prec, rtol=1e-8, maxit=100, raise_on_fail=False)
            storage16["%s/%s" % (prec, w["name"])] = {
                "iterations": info["iterations"], "relres": info["relres"], "status": info["status"],
                "seconds": info["seconds"], "converged": info["status"] == 0}
            log("%s-preconditioned %s: its %d relres %.2e" % (prec, forms[0], info["iterations"], info["relres"]))
        import iss_inputs as _inp
        ws = _inp.workload("sphere_3d")
        Ps = Problem.from_workload(ws, outer="fgmres", restart=150, coarse_mu="average", nu1=args.nu, nu2=args.nu,
                                   nu_inc=args.nu_inc, omega=args.omega, coarse_form=coarse_form,
                                   mid_form=mid_form, cycles=args.cycles)
        bs = torch.zeros(Ps.vector_size(), dtype=torch.float64, device=dev)
        Ps.rhs_buoyancy(bs, ws["buoyant"])
        xs64 = torch.zeros_like(bs)
        Ps.solve(forms[0], xs64, bs, rtol=1e-8, maxit=200, raise_on_fail=False)
        Ns = Ps.num_vertices()
        for prec in ("fp64", "fp32", "bf16", "fp16"):
            xs = torch.zeros_like(bs)
            Ps.solve(forms[0], xs, bs, prec=prec, rtol=1e-8, maxit=200, raise_on_fail=False)
            xs.zero_()
            torch.cuda.synchronize()
            t = time.perf_counter()
            info = Ps.solve(forms[0], xs, bs, prec=prec, rtol=1e-8, maxit=200, raise_on_fail=False)
            torch.cuda.synchronize()
            errs = []
            for f in range(4):
                a_, c_ = xs[f * Ns:(f + 1) * Ns], xs64[f * Ns:(f + 1) * Ns]
                if f == 3:
                    a_, c_ = a_ - a_.mean(), c_ - c_.mean()
                errs.append(float(torch.linalg.norm(a_ - c_) / torch.linalg.norm(c_)))
            storage16["%s/sphere_3d 65^3 mu 1e3" % prec] = {
                "iterations": info["iterations"], "relres": info["relres"], "status": info["status"],
                "seconds": time.perf_counter() - t, "converged": info["status"] == 0,
                "rel_error_per_field_vs_fp64": errs}
        Ps.close()
        log("16-bit storage: %s" % {k: (v["iterations"], v["converged"]) for k, v in storage16.items()})

    learned = None
    if not args.no_learned:
        learned = learned_report()

    # asymptotic rate of the stationary cycle per form (Sec. 5: residual
    # reduction per cycle of the homogeneous problem, rescaled every cycle)
    rates = None
    if args.rate_iters > 0:
        import iss_inputs as _inp
        rates = {}
        x0 = torch.from_numpy(_inp.random_vector(w["dim"], w["n"], seed=7)).to(dev)
        for form in forms:
            xr0 = x0.clone()
            hist = P.asymptotic_rate(form, xr0, iters=args.rate_iters)
            rates[form] = {"rate": hist[-1], "mean_last_20": sum(hist[-20:]) / len(hist[-20:]),
                           "iterations": args.rate_iters}
        log("asymptotic rates: %s" % rates)

    apply_gbs = {}
    smooth_ms = {}
    if not args.quick:
        xr = torch.rand(nvec, dtype=torch.float64, device=dev)
        y = torch.empty_like(xr)
        for form in ("interface", "strain", "gradient"):
            for block, bpv in (("velocity", 6 * 8 + 1), ("full", 8 * 8 + 1)):
                ms = event_time(lambda: P.apply(form, xr, y, block=block), 20)
                apply_gbs["%s/%s" % (form, block)] = {"ms": ms, "GBs": bpv * N / ms / 1e6,
                                                       "bytes_per_vertex": bpv}
        for form in forms:
            xs = torch.zeros_like(b)
            P.smooth(form, xs, b, 1)
            phase, step = P.smooth_timed(form, xs, b, 5)
            smooth_ms[form] = {"velocity_colour_phase_ms": phase, "step_ms": step}
        log("apply GB/s: %s" % {k: round(v["GBs"], 1) for k, v in apply_gbs.items()})
        # stabilised P1-P0 (Sec. 3) on the same lattice: K x with one pressure
        # per element and the interior-penalty form, and the flux post-process
        ne = P.num_elements()
        xp = torch.rand(P.p1p0_size(), dtype=torch.float64, device=dev)
        yp = torch.empty_like(xp)
        fl = torch.empty(ne * (w["dim"] + 1), dtype=torch.float64, device=dev)
        for form in ("interface", "strain"):
            ms = event_time(lambda: P.p1p0_apply(form, xp, yp), 10)
            # read u (3 fields), p (one per element), element and vertex
            # phases; write K x: 3 * 8 + 8 ne / N + ne / N + 1 + 3 * 8 + 8 ne / N
            bpv = 49 + 17 * ne / N
            apply_gbs["p1p0/%s/full" % form] = {"ms": ms, "GBs": bpv * N / ms / 1e6, "bytes_per_vertex": bpv}
        ms = event_time(lambda: P.p1p0_flux(xp, fl), 10)
        bpv = 24 + 9 * ne / N + 4 * 8 * ne / N
        apply_gbs["p1p0/flux"] = {"ms": ms, "GBs": bpv * N / ms / 1e6, "bytes_per_vertex": bpv}
        del xp, yp, fl
        log("P1-P0: %s" % {k: (round(v["ms"], 3), round(v["GBs"], 1)) for k, v in apply_gbs.items()
                           if k.startswith("p1p0")})
        log("smoothing (HIP events): %s" % smooth_ms)

    # the paper's own configuration: a_tr (the call's form) on every level
    # but the coarsest, which takes the strain form (Sec. 5), for the record
    paper_cfg = None
    if not args.no_paper_config and "interface" in forms:
        P.close()
        torch.cuda.empty_cache()
        Pp = Problem.from_workload(w, outer=args.outer, omega=args.omega, restart=args.restart,
                                   coarse_mu=args.coarse_mu, nu1=args.nu, nu2=args.nu, nu_inc=args.nu_inc,
                                   coarse_form="strain", mid_form=None, cycles=args.cycles, coarse_rhs_mod=True)
        x.zero_()
        info = Pp.solve("interface", x, b, rtol=1e-8, maxit=150, raise_on_fail=False)
        paper_cfg = {"config": "a_tr on every level but the coarsest (strain form there, momentum right-hand "
                               "side modified with B^T M^-1 r_2), otherwise the headline solver, maxit 150",
                     "iterations": info["iterations"], "relres": info["relres"], "status": info["status"],
                     "seconds": info["seconds"]}
        log("paper configuration: its %d relres %.2e status %d" % (info["iterations"], info["relres"],
                                                                   info["status"]))
        Pp.close()

    columns = None
    if not args.no_columns:
        P.close()
        torch.cuda.empty_cache()
        columns = columns_report(args.rate_iters)

    main_form = forms[0]
    value = results[main_form]["seconds"]
    # Roofline of the dominant kernel, the bulk velocity Gauss-Seidel colour
    # phase (k_gs_vel_s; the largest kernel-time share of a solve), on the
    # method's algorithmic bytes: a velocity Gauss-Seidel sweep over all
    # colours must read u (3 fields), f (3) and p (for B^T p) and write u (3):
    # 10 values of 8 B plus the phase byte = 81 B per vertex per sweep, so
    # one of the d+1 colour-phase launches of a sweep is charged 81/(d+1) B
    # per interior vertex.  The whole smoothing step is charged the
    # symmetric sweep (162 B) plus the pressure Uzawa step (u, p, g read,
    # p written, phase: 49 B) = 211 B per interior vertex.
    roof = roof_step = roof_phase = None
    if smooth_ms:
        n_int = (w["n"] - 1) ** w["dim"]
        bytes_launch = 81.0 / (w["dim"] + 1) * n_int
        ms = smooth_ms[main_form]["velocity_colour_phase_ms"]
        ach = bytes_launch / (ms * 1e-3) / 1e9
        roof = {"bound": "hbm",
                "kernel": "k_gs_vel_s (%s form, bulk velocity colour phase, finest level, FP64)" % main_form,
                "algorithmic_bytes_per_launch": bytes_launch, "bytes_per_vertex_per_sweep": 81,
                "ms_per_launch": ms, "achieved": ach, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": ach / PEAK_HBM_GBS, "traffic": measured_traffic("k_gs_vel_s", main_form)}
        # the same launch charged what one colour phase on its own must
        # move: every colour neighbours every other in the Kuhn stencil, so
        # all of u is read (24 B per vertex), besides the own colour's g
        # and phase byte, and the own colour's u is written (24 + (24 + 1 +
        # 24) / (d + 1) B per interior vertex in 3D)
        M = w["dim"] + 1
        phase_bytes = (8.0 * w["dim"] + (16.0 * w["dim"] + 1) / M) * n_int
        roof_phase = {"bound": "hbm", "what": "the same launch, bytes a single colour phase must move",
                      "bytes_per_launch": phase_bytes, "ms_per_launch": ms,
                      "achieved": phase_bytes / (ms * 1e-3) / 1e9, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                      "frac": phase_bytes / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS}
        step_bytes = 211.0 * n_int
        st = smooth_ms[main_form]["step_ms"]
        roof_step = {"bound": "hbm", "what": "one Uzawa smoothing step, finest level, FP64, all kernels",
                     "algorithmic_bytes": step_bytes, "bytes_per_vertex": 211, "ms": st,
                     "achieved": step_bytes / (st * 1e-3) / 1e9, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": step_bytes / (st * 1e-3) / 1e9 / PEAK_HBM_GBS}
    cpu = None
    if not args.no_cpu:
        try:
            cpu = cpu_baseline(w, results[main_form]["iterations"], args.omega, args.nu, args.restart,
                               args.nu_inc, args.cycles, mid_form, coarse_form)
        except Exception as e:   # reported, never silently replaced
            cpu = {"error": str(e)[-300:]}
        if args.cpu_full and "error" not in cpu:
            try:
                cpu["full_solves"] = full_solves(Problem, args, mid_form, coarse_form, forms)
            except Exception as e:
                cpu["full_solves"] = {"error": str(e)[-300:]}
    out = {
        "metric": "s to 1e-8 rel. residual & stencil GB/s: decoupled vs strain form, 1 MI355X",
        "value": value, "unit": "s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": value * 1e3, "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "%s: %d^3 vertices, %d unknowns, %d spheres mu_in %.0e, %d interface "
                               "vertices" % (w["name"], w["n"] + 1, nvec, len(w["inclusions"]),
                                             w["mu"][1], nif),
                   "solver": "%s(%d), preconditioner %d stationary Uzawa V(%d,%d) cycles +%d steps per "
                             "coarser level, omega %.2f, coarse viscosity %s, levels below the finest in the "
                             "%s form, coarsest in the %s form"
                             % (args.outer, args.restart, args.cycles, args.nu, args.nu, args.nu_inc, args.omega,
                                args.coarse_mu, args.mid_form, args.coarse_form),
                   "parallelism": "single GPU"},
        "forms": results,
        "strain_over_interface": (results["strain"]["seconds"] / results["interface"]["seconds"])
        if "strain" in results and "interface" in results else None,
        "mixed_precision": fp32,
        "storage_16bit": storage16,
        "learned_correction": learned,
        "apply": apply_gbs,
        "smooth_step_ms": smooth_ms,
        "paper_configuration": paper_cfg,
        "viscosity_columns": columns,
        "asymptotic_rate": rates,
        "roofline": roof,
        "roofline_smoothing_step": roof_step,
        "roofline_colour_phase_minimum": roof_phase,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
