"""Training and evaluation of the learned interface-band correction.

Data come from the solver itself.  For every seeded inclusion geometry of the
workload ``learned_3d`` (65^3, 1-16 spheres, radii U[0.05, 0.2], contrast
10^U[1, 4]) the FP64 solution x* of the buoyancy problem is computed with
FGMRES to 1e-11; then `snapshots` stationary steps x_{k+1} = x_k + z_k,
z_k = V(b - K x_k) are taken and after each V-cycle the pair

    input  r' = r_k - K z_k            (the residual the V-cycle leaves)
    target e' = x* - x_k - z_k         (= K^{-1} r', the error it leaves)

is stored compactly: the network input on the band (8 channels, BF16) and
the target on the band in the network's output units (4 channels, FP32).
Every vector operation runs in the library (residuals, V-cycles, iss_axpby,
the band feature and target kernels); torch only provides memory.

Training minimises the mean squared error of the output against the target
(the loss of the oracle's ``mse``) with Adam, one pair per step, the forward
and backward passes in the library's BF16 MFMA kernels.  A validation loss on
separate seeds is logged each epoch.  The gain test solves held-out
geometries with FGMRES, plain and with the correction attached (the
safeguard keeps a correction only if it lowers the residual), and reports
iterations and time; a gain of zero or less is reported as it is.

Seeds: training 0..999 (10 snapshots each: 10^4 pairs), validation
1000..1099, held out 100000..100049.

Usage:
    python -m paper_1604_07994_amd.learned --out weights.npz
"""
import argparse
import json
import os
import sys
import time

import numpy as np

from .binding import BandNet, Problem, adam_step

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import iss_inputs  # noqa: E402  (seeded workload descriptions, repo root)

SOLVER = dict(outer="fgmres", omega=0.6, nu1=3, nu2=3, restart=60, coarse_mu="average",
              coarse_form="strain", mid_form="strain")
FORM = "interface"


def _workload(seed, levels):
    return iss_inputs.workload("learned_3d", seed=seed, levels=levels)


def buoyancy_rhs(P, w):
    import torch
    b = torch.zeros(P.vector_size(), dtype=torch.float64, device="cuda")
    P.rhs_buoyancy(b, w["buoyant"])
    return b


def generate(seeds, levels=6, snapshots=10, log=print):
    """Networks (one per geometry, each holding its band) and the stored
    pairs [(network index, input M x 8 BF16 bits, target M x 4 FP32)]."""
    import torch
    nets, pairs, skipped = [], [], 0
    t0 = time.time()
    for q, s in enumerate(seeds):
        w = _workload(s, levels)
        P = Problem.from_workload(w, **SOLVER)
        net = BandNet(P)
        if net.band_size == 0:
            skipped += 1
            net.close()
            P.close()
            continue
        b = buoyancy_rhs(P, w)
        xs = torch.zeros_like(b)
        P.solve(FORM, xs, b, rtol=1e-11, maxit=600, raise_on_fail=False)
        x = torch.zeros_like(b)
        r, rp, z, e = (torch.zeros_like(b) for _ in range(4))
        for _ in range(snapshots):
            P.residual(FORM, x, b, r)                  # r = b - K x
            P.axpby(0.0, r, 0.0, z)                    # z = 0
            P.vcycle(FORM, z, r)                       # z = V(r)
            P.residual(FORM, z, r, rp)                 # r' = r - K z
            P.axpby(1.0, xs, 0.0, e)                   # e' = x* - x - z
            P.axpby(-1.0, x, 1.0, e)
            P.axpby(-1.0, z, 1.0, e)
            net.features(rp)
            feat = torch.empty(net.band_size * 8, dtype=torch.int16, device="cuda")
            tgt = torch.empty(net.band_size * 4, dtype=torch.float32, device="cuda")
            net.save_input(feat)
            net.targets(e, tgt)
            pairs.append((len(nets), feat, tgt))
            P.axpby(1.0, z, 1.0, x)                    # x += z
        nets.append(net)
        P.close()                                      # the network outlives its problem
        if (q + 1) % 50 == 0:
            log("generated %d pairs from %d geometries (%d seeds) in %.1f s"
                % (len(pairs), len(nets), q + 1, time.time() - t0))
    return nets, pairs, {"geometries": len(nets), "pairs": len(pairs), "no_band": skipped,
                         "seconds": time.time() - t0}


def initial_weights(seed=0):
    """He-style initialisation of the hidden layers; the output layer starts
    near zero, so training starts from (almost) no correction."""
    rng = np.random.default_rng(seed)
    sizes = [(16, 8), (16, 16), (4, 16)]
    return np.concatenate([rng.normal(size=co * ci * 27) * np.sqrt(2.0 / (ci * 27)) * (1e-3 if co == 4 else 1.0)
                           for co, ci in sizes]).astype(np.float32)


def mean_loss(nets, pairs, wt, g):
    """Mean MSE over stored pairs (the forward and loss of the library)."""
    tot = 0.0
    for k, feat, tgt in pairs:
        net = nets[k]
        net.set_weights(wt)
        net.load_input(feat)
        net.forward()
        tot += net.backward(tgt, g)
    return tot / max(1, len(pairs))


def train(nets, pairs, val_nets, val_pairs, epochs=8, lr=1e-3, seed=0, log=print):
    import torch
    rng = np.random.default_rng(seed)
    wt = torch.from_numpy(initial_weights(seed)).cuda()
    m, v, g = torch.zeros_like(wt), torch.zeros_like(wt), torch.empty_like(wt)
    step, hist, val = 0, [], []
    t0 = time.time()
    val.append(mean_loss(val_nets, val_pairs, wt, g))
    log("epoch -1 validation loss %.5f" % val[-1])
    for ep in range(epochs):
        tot = 0.0
        for idx in rng.permutation(len(pairs)):
            k, feat, tgt = pairs[idx]
            net = nets[k]
            net.set_weights(wt)
            net.load_input(feat)
            net.forward()
            tot += net.backward(tgt, g)
            step += 1
            adam_step(wt, m, v, g, lr, step)
        hist.append(tot / len(pairs))
        val.append(mean_loss(val_nets, val_pairs, wt, g))
        log("epoch %d training loss %.5f validation loss %.5f (%.1f s)" % (ep, hist[-1], val[-1], time.time() - t0))
    return wt.cpu().numpy(), {"epochs": epochs, "lr": lr, "steps": step, "train_loss": hist,
                              "validation_loss": val, "train_seconds": time.time() - t0}


def evaluate(weights, seeds, levels=6, rtol=1e-8, log=print):
    """FGMRES iterations and time to rtol on held-out geometries, plain vs
    with the band correction attached."""
    import torch
    rows = []
    wt = torch.from_numpy(np.asarray(weights, dtype=np.float32)).cuda()
    for s in seeds:
        w = _workload(s, levels)
        P = Problem.from_workload(w, **SOLVER)
        net = BandNet(P)
        b = buoyancy_rhs(P, w)
        res = {}
        for mode in ("plain", "net"):
            net.attach(mode == "net")
            if mode == "net":
                net.set_weights(wt)
            x = torch.zeros_like(b)
            P.solve(FORM, x, b, rtol=rtol, maxit=600, raise_on_fail=False)   # warm
            x = torch.zeros_like(b)
            info = P.solve(FORM, x, b, rtol=rtol, maxit=600, raise_on_fail=False)
            res[mode] = {"iterations": info["iterations"], "seconds": info["seconds"],
                         "relres": info["relres"], "accepted": info["net_accepted"],
                         "rejected": info["net_rejected"]}
        net.attach(False)
        row = {"seed": s, "spheres": len(w["inclusions"]), "contrast": w["mu"][1], "band": net.band_size,
               **{"%s_%s" % (m_, k): v for m_ in res for k, v in res[m_].items()}}
        log(json.dumps(row))
        rows.append(row)
        net.close()
        P.close()
    return rows


def summarise(rows):
    pi = np.array([r["plain_iterations"] for r in rows], float)
    ni = np.array([r["net_iterations"] for r in rows], float)
    ps = np.array([r["plain_seconds"] for r in rows], float)
    ns = np.array([r["net_seconds"] for r in rows], float)
    return {"geometries": len(rows),
            "plain_iterations_mean": float(pi.mean()), "net_iterations_mean": float(ni.mean()),
            "plain_seconds_mean": float(ps.mean()), "net_seconds_mean": float(ns.mean()),
            "iteration_gain_mean": float((pi - ni).mean()), "time_gain_mean": float((ps - ns).mean()),
            "fewer_iterations": int((ni < pi).sum()), "more_iterations": int((ni > pi).sum())}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--levels", type=int, default=6)
    ap.add_argument("--train-seeds", type=int, default=1000)
    ap.add_argument("--val-seeds", type=int, default=100)
    ap.add_argument("--test-seeds", type=int, default=50)
    ap.add_argument("--snapshots", type=int, default=10)
    ap.add_argument("--epochs", type=int, default=8)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--stage", choices=["all", "train", "evaluate"], default="all",
                    help="train: data and training only (writes the weights and the log); evaluate: the "
                         "held-out comparison with the weights in --out, added to its log")
    args = ap.parse_args()
    log = lambda s: print(s, flush=True)
    log_path = args.out.rsplit(".", 1)[0] + ".json"
    test = list(range(100000, 100000 + args.test_seeds))
    if args.stage == "evaluate":
        weights = np.load(args.out, allow_pickle=False)["weights"]
        with open(log_path) as f:
            meta = json.load(f)
        rows = evaluate(weights, test, args.levels, log=log)
        meta.update({"test_seeds": test, "evaluation": rows, "summary": summarise(rows)})
        with open(log_path, "w") as f:
            json.dump(meta, f, indent=1)
        log("summary " + json.dumps(meta["summary"]))
        return
    nets, pairs, gen = generate(list(range(args.train_seeds)), args.levels, args.snapshots, log=log)
    log("training data: %s" % gen)
    vnets, vpairs, vgen = generate(list(range(1000, 1000 + args.val_seeds)), args.levels, args.snapshots, log=log)
    log("validation data: %s" % vgen)
    weights, meta = train(nets, pairs, vnets, vpairs, args.epochs, args.lr, log=log)
    for n_ in nets + vnets:
        n_.close()
    meta.update({"levels": args.levels, "snapshots": args.snapshots, "training_data": gen,
                 "validation_data": vgen, "train_seeds": [0, args.train_seeds - 1],
                 "validation_seeds": [1000, 1000 + args.val_seeds - 1], "solver": SOLVER})
    np.savez(args.out, weights=weights)
    if args.stage == "all":
        rows = evaluate(weights, test, args.levels, log=log)
        meta.update({"test_seeds": test, "evaluation": rows, "summary": summarise(rows)})
        log("summary " + json.dumps(meta["summary"]))
    with open(log_path, "w") as f:
        json.dump(meta, f, indent=1)


if __name__ == "__main__":
    main()
