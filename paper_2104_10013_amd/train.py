"""Train one of the workloads with the fused step and report the loss history
and the relative L2 error of the stitched solution (Eq. FSol) against the
exact solution on the workload's evaluation grid.

    python -m paper_2104_10013_amd.train --workload c1_cpinn_poisson --steps 100

Prints one JSON line per report and a final summary line.  For the inverse
problem the error of the inferred conductivity K is reported as well.
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np
import torch

from . import ddpinn, workloads as W


def rel_l2(u, exact):
    return float(np.linalg.norm(u - exact) / np.linalg.norm(exact))


def stitched_errors(pb, prob):
    out = pb.eval(prob.eval_xy, prob.eval_owner).cpu().numpy().astype(np.float64)
    ex = np.asarray(prob.eval_exact, np.float64)
    if prob.pde == W.PDE_DIFFUSION2D_INV:
        return {"u": rel_l2(out[:, 0], ex[:, 0]), "K": rel_l2(out[:, 1], ex[:, 1])}
    if prob.d_out == 3:   # Navier-Stokes (u, v, p); the pressure is fixed by its data up to noise
        return {"u": rel_l2(out[:, 0], ex[:, 0]), "v": rel_l2(out[:, 1], ex[:, 1]), "p": rel_l2(out[:, 2], ex[:, 2])}
    return {"u": rel_l2(out[:, 0], ex[:, 0])}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="c1_cpinn_poisson", choices=sorted(W.WORKLOADS))
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--scale", type=float, default=1.0, help="point-count scale of the workload")
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--report-every", type=int, default=0, help="0: only at the end")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--lr", type=float, default=None, help="Adam learning rate of every subdomain (default: the workload's)")
    ap.add_argument("--loss-w", type=float, nargs=4, default=None, metavar=("W_U", "W_F", "W_I", "W_4"),
                    help="loss weights of every subdomain (data, residual, average, flux or residual continuity)")
    args = ap.parse_args(argv)

    prob = W.make_problem(args.workload, seed=args.seed, scale=args.scale)
    for sd in prob.subdomains:
        if args.lr is not None:
            sd.lr = args.lr
        if args.loss_w is not None:
            sd.loss_w = tuple(args.loss_w)
    pb = ddpinn.Problem(prob, fused=True)
    if not args.no_autotune:
        pb.autotune(iters=5)
    init = stitched_errors(pb, prob)
    every = args.report_every if args.report_every > 0 else args.steps
    done = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    while done < args.steps:
        n = min(every, args.steps - done)
        lt = pb.step(n)
        done += n
        pb.sync()
        J = lt[:, 0].cpu().numpy().astype(np.float64)
        print(json.dumps({"step": done, "sum_J": float(J.sum()), "max_J": float(J.max())}), flush=True)
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    final = stitched_errors(pb, prob)
    print(json.dumps({"workload": args.workload, "seed": args.seed, "scale": args.scale, "steps": args.steps,
                      "lr": args.lr, "loss_w": args.loss_w,
                      "rel_l2_init": init, "rel_l2_final": final, "train_s": secs,
                      "steps_per_s": args.steps / secs}), flush=True)
    pb.close()


if __name__ == "__main__":
    main()
