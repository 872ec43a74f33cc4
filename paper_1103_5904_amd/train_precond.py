"""Train the learned preconditioner on seeded synthetic problems and write
its weights (python -m paper_1103_5904_amd.train_precond --out FILE).

Problems: 128^3 blob phantoms on [-1.5, 1.5]^3 seen by the 28 EUVI-like
views at 256x256, 1% noise, lambda 1e-2 (tomo_synth.learned), seeds 1000 +
k.  Pairs come from the library's plain CG (iterates 0..39, x* from CG to
1e-6 or 300 iterations): 50 problems give 2000 pairs.  The fit minimises the
energy-norm error of the network's correction with the library's network
gradient, projector and Adam kernels.  Held-out problems (seeds 2000 + k)
then time plain CG and flexible CG with the network to relative residual
1e-3.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import tomo_synth as ts  # noqa: E402

from . import precond as pc  # noqa: E402
from . import tomo as _t  # noqa: E402


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.join(os.path.dirname(__file__), "precond_weights.npz"))
    ap.add_argument("--train-seeds", type=int, default=50, help="problems, seeds 1000, 1001, ...")
    ap.add_argument("--records", type=int, default=40)
    ap.add_argument("--epochs", type=int, default=2)
    ap.add_argument("--lr", type=float, default=3e-4)
    ap.add_argument("--lr-final", type=float, default=3e-5)
    ap.add_argument("--init", default=None,
                    help="start from these weights (.npz) instead of the fitted linear filter")
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--npix", type=int, default=256)
    ap.add_argument("--eval-seeds", type=int, default=3, help="held-out problems, seeds 2000, ...")
    args = ap.parse_args(argv)
    torch.cuda.set_device(0)
    log = lambda s: print(s, flush=True)  # noqa: E731
    t0 = time.perf_counter()
    ins, tgs = [], []
    dg = None
    for k in range(args.train_seeds):
        wl = ts.learned(1000 + k, n=args.n, npix=args.npix)
        dg = dg or _t.DeviceGeometry(wl.geom)  # same views and box for every seed
        y = pc.noisy_data(dg, torch.as_tensor(wl.x.astype(np.float32)).cuda(), wl.noise_rel,
                          wl.noise_seed)
        a, b = pc.solve_pairs(dg, y, wl.lam_r, k_record=args.records)
        ins.append(a)
        tgs.append(b)
        if (k + 1) % 10 == 0:
            log(f"pairs from {k + 1} problems ({time.perf_counter() - t0:.1f} s)")
    inputs = torch.cat(ins)
    targets = torch.cat(tgs)
    del ins, tgs
    t1 = time.perf_counter()
    h = pc.fit_linear_filter(pc.NormalOperator(dg, wl.lam_r), inputs[0:args.records:4])
    log("linear filter fit (kz, ky, kx):\n" + np.array2string(h, precision=4, suppress_small=True))
    lin = pc.linear_filter_params(h)
    if args.init:
        init = pc.load(args.init).cpu().numpy().astype(np.float64)
    else:
        init = lin + 1e-3 * np.random.default_rng(0).normal(size=lin.shape) * (lin == 0)
    params, losses = pc.train(dg, wl.lam_r, inputs, targets, epochs=args.epochs, lr=args.lr,
                              lr_final=args.lr_final, log=log, init=init)
    t_train = time.perf_counter() - t1
    lin_d = torch.as_tensor(lin.astype(np.float32)).cuda()
    del inputs, targets
    # held-out evaluation
    evals = []
    for k in range(args.eval_seeds):
        wl = ts.learned(2000 + k, n=args.n, npix=args.npix)
        dg = _t.DeviceGeometry(wl.geom)
        y = pc.noisy_data(dg, torch.as_tensor(wl.x.astype(np.float32)).cuda(), wl.noise_rel,
                          wl.noise_seed)
        pc.time_to_tolerance(dg, y, wl.lam_r, 1e-3, None)  # warm-up
        tp, rp = pc.time_to_tolerance(dg, y, wl.lam_r, 1e-3, None, reps=3)
        tl, rl = pc.time_to_tolerance(dg, y, wl.lam_r, 1e-3, params, reps=3)
        tf, rf = pc.time_to_tolerance(dg, y, wl.lam_r, 1e-3, lin_d, reps=3)
        evals.append({"seed": 2000 + k, "plain_ms": tp, "plain_iters": rp["iters"],
                      "learned_ms": tl, "learned_iters": rl["iters"], "fell_back": rl["fell_back"],
                      "learned_true_rel_res": rl["true_rel_res"], "filter_ms": tf,
                      "filter_iters": rf["iters"]})
        log(json.dumps(evals[-1]))
    meta = {"train_seeds": args.train_seeds, "records": args.records, "epochs": args.epochs,
            "lr": args.lr, "lr_final": args.lr_final, "init": args.init, "n": args.n, "npix": args.npix,
            "filter": h.ravel().tolist(), "losses": losses, "train_s": t_train, "pairs_s": t1 - t0, "eval": evals}
    pc.save(args.out, params, meta)
    log(f"wrote {args.out}")
    print(json.dumps({"eval": evals, "losses": losses, "train_s": t_train}), flush=True)


if __name__ == "__main__":
    main()
