"""Train the unrolled PSCA network's step sizes on generated instances.

    python -m paper_2503_15259_amd.train_net --variant MAP-UR --K 20 --steps 200 --batch 8 \\
        --out paper_2503_15259_amd/data/net_MAP-UR_K20.json

Training instances are instance i of the "net" workload (seeds [3, i]);
validation uses seeds from 10^6 on, disjoint from training.  The step sizes
kept are those of the best validation loss seen (checked 20 times during
training), and the detection threshold is the one minimising the validation
error rate.
Every forward and backward pass runs in the HIP kernels: a minibatch goes
through one psca_detect_batch launch with every iterate recorded and one
psca_layer_backward_batch launch per layer, validation through
psca_net_forward; Adam on the K step sizes, projected to [0, 1].
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--variant", default="MAP-UR", choices=["ML-K", "MAP-K", "ML-UD", "MAP-UR"])
    ap.add_argument("--K", type=int, default=20)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--val", type=int, default=16)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--N", type=int, default=1000)
    ap.add_argument("--L", type=int, default=64)
    ap.add_argument("--M", type=int, default=128)
    ap.add_argument("--p", type=float, default=0.1)
    ap.add_argument("--eps", type=float, default=0.01)
    ap.add_argument("--out", required=True)
    args = ap.parse_args()

    import torch
    from . import instances as I
    from . import net as NET
    from . import psca as P

    dev = torch.device("cuda", 0)
    variant = P.VARIANTS[args.variant]
    wid = I.WORKLOAD_IDS["net"]
    ctx = P.Context(0)

    def load(index):
        inst = I.make_instance(wid, index, args.N, args.L, args.M, args.p)
        S = P.colmajor(torch.from_numpy(inst.S.astype(np.complex64)).to(dev))
        Y = P.colmajor(torch.from_numpy(inst.Y.astype(np.complex64)).to(dev))
        g = torch.from_numpy(inst.g.astype(np.float32)).to(dev)
        kw = dict(variant=variant, iters=args.K, sigma2=inst.sigma2, M=inst.M, d_lo=inst.d_lo, d_hi=inst.d_hi,
                  pl_c0=inst.pl_c0, pl_beta=inst.pl_beta, eps=args.eps)
        if variant in (P.ML_K, P.MAP_K):
            kw["g"] = g
        if variant == P.MAP_K:
            kw["p"] = torch.full((inst.N,), inst.p, dtype=torch.float32, device=dev)
        alpha = torch.from_numpy(inst.alpha.astype(np.float32)).to(dev)
        return P.sample_cov(Y, ctx=ctx), S, P.Params(**kw), alpha, g

    model = NET.PscaNet(args.K, load(0)[2], ctx=ctx)
    opt = torch.optim.Adam(model.parameters(), lr=args.lr)
    val = [load(10 ** 6 + i) for i in range(args.val)]

    def val_loss():
        with torch.no_grad():
            tot = 0.0
            for Sh, S, prm, alpha, g in val:
                tot += float(NET.bce(model(Sh, S, prm), alpha, g, model.known))
            model.status.check()
            return tot / len(val)

    history = [{"step": 0, "val_loss": val_loss()}]
    best_val, best_rho, best_step = history[0]["val_loss"], model.rho.detach().clone(), 0
    t0 = time.perf_counter()
    next_index = 0
    for step in range(1, args.steps + 1):
        batch = [load(next_index + b) for b in range(args.batch)]
        next_index += args.batch
        loss = NET.train_step(model, opt, batch)
        if step % max(1, args.steps // 20) == 0 or step == args.steps:
            history.append({"step": step, "train_loss": loss, "val_loss": val_loss(),
                            "seconds": round(time.perf_counter() - t0, 2)})
            print(json.dumps(history[-1]), flush=True)
            if history[-1]["val_loss"] < best_val:   # keep the step sizes of the best validation loss
                best_val, best_rho, best_step = history[-1]["val_loss"], model.rho.detach().clone(), step
    with torch.no_grad():
        model.rho.copy_(best_rho)
    with torch.no_grad():
        scores, truths = [], []
        for Sh, S, prm, alpha, g in val:
            x = model(Sh, S, prm)
            scores.append(x if model.known else x / g)
            truths.append(alpha)
        model.status.check()
        theta = NET.choose_threshold(scores, truths)
    out = {"variant": args.variant, "K": args.K, "rho": [float(r) for r in model.rho.detach().cpu()],
           "best_step": best_step, "best_val_loss": best_val, "theta": theta, "threshold_on": "alpha~" if model.known else "gamma~/g",
           "train": {"steps": args.steps, "batch": args.batch, "lr": args.lr, "instances": next_index,
                     "N": args.N, "L": args.L, "M": args.M, "p": args.p, "eps": args.eps,
                     "seeds": "training: [3, i] for i < instances; validation: [3, 10^6 + i]"},
           "history": history}
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    with open(args.out, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", args.out, "theta", theta, "rho", [round(r, 4) for r in out["rho"]], flush=True)


if __name__ == "__main__":
    sys.exit(main())
