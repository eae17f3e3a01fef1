"""Train the unrolled PSCA network's step sizes on generated instances.

    python -m paper_2503_15259_amd.train_net --variant MAP-UR --K 20 --batch 512 --steps 400 \\
        --pool 4096 --lr 1e-3 --out paper_2503_15259_amd/data/net_MAP-UR_K20.json

Training instances are instance i of the "net" workload (seeds [3, i]) at the
requested sizes; with --pool P a pool of P distinct instances is drawn once
(in parallel host processes) and every step takes a seeded random minibatch
from it, else every step draws fresh instances.  Validation uses seeds from
10^6 on, disjoint from training.  Every --val-every steps the validation
loss is evaluated; the step sizes of the best validation loss are kept and
training stops once --patience evaluations in a row have not improved it
(the paper trains until the validation loss stops improving).  The step
sizes start from the schedule rho_{k+1} = rho_k (1 - rho_k / 2), rho_0 = 0.5
(Sec. VI), or with --init from those of a network trained before (a JSON file
written by this script; its "rho" must have K entries).  The detection
threshold is the one minimising the validation error rate.
Every forward and backward pass runs in the HIP kernels: a minibatch goes
through one psca_detect_batch launch with every iterate recorded and one
psca_layer_backward_batch launch per layer, validation through
psca_net_forward; Adam on the K step sizes, projected to [0, 1].
"""
from __future__ import annotations

import argparse
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np


def _draw(args):
    """One seeded instance as the arrays the GPU receives (host process)."""
    os.environ["OPENBLAS_NUM_THREADS"] = "1"
    from . import instances as I
    wid, index, N, L, M, p = args
    inst = I.make_instance(wid, index, N, L, M, p)
    return (index, inst.S.astype(np.complex64), inst.Y.astype(np.complex64), inst.g.astype(np.float32),
            inst.alpha.astype(np.float32), float(inst.sigma2), int(inst.M), float(inst.d_lo), float(inst.d_hi),
            float(inst.pl_c0), float(inst.pl_beta))


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--variant", default="MAP-UR", choices=["ML-K", "MAP-K", "ML-UD", "MAP-UR"])
    ap.add_argument("--K", type=int, default=20)
    ap.add_argument("--steps", type=int, default=200, help="largest number of Adam steps")
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--pool", type=int, default=0, help="distinct training instances drawn once (0: fresh each step)")
    ap.add_argument("--val", type=int, default=16)
    ap.add_argument("--val-every", type=int, default=10)
    ap.add_argument("--patience", type=int, default=0, help="stop after this many evaluations without improvement")
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--N", type=int, default=1000)
    ap.add_argument("--L", type=int, default=64)
    ap.add_argument("--M", type=int, default=128)
    ap.add_argument("--p", type=float, default=0.1)
    ap.add_argument("--eps", type=float, default=0.01)
    ap.add_argument("--workers", type=int, default=16, help="host processes drawing instances")
    ap.add_argument("--init", default="", help="start from the step sizes of this trained-network JSON file")
    ap.add_argument("--out", required=True)
    args = ap.parse_args()

    import torch
    from . import instances as I
    from . import metrics
    from . import net as NET
    from . import psca as P

    dev = torch.device("cuda", 0)
    variant = P.VARIANTS[args.variant]
    wid = I.WORKLOAD_IDS["net"]
    ctx = P.Context(0)

    def upload(arrs):
        _, S, Y, g, alpha, sigma2, M, d_lo, d_hi, pl_c0, pl_beta = arrs
        S = P.colmajor(torch.from_numpy(S).to(dev))
        Yd = P.colmajor(torch.from_numpy(Y).to(dev))
        g = torch.from_numpy(g).to(dev)
        kw = dict(variant=variant, iters=args.K, sigma2=sigma2, M=M, d_lo=d_lo, d_hi=d_hi,
                  pl_c0=pl_c0, pl_beta=pl_beta, eps=args.eps)
        if variant in (P.ML_K, P.MAP_K):
            kw["g"] = g
        if variant == P.MAP_K:
            kw["p"] = torch.full((S.shape[1],), args.p, dtype=torch.float32, device=dev)
        return P.sample_cov(Yd, ctx=ctx), S, P.Params(**kw), torch.from_numpy(alpha).to(dev), g

    def draw(indices):
        tasks = [(wid, i, args.N, args.L, args.M, args.p) for i in indices]
        workers = max(1, min(args.workers, len(tasks)))
        if workers == 1:
            return [upload(_draw(t)) for t in tasks]
        out = []
        saved = {k: os.environ.get(k) for k in ("OPENBLAS_NUM_THREADS", "OMP_NUM_THREADS")}
        os.environ.update(OPENBLAS_NUM_THREADS="1", OMP_NUM_THREADS="1")   # read by the workers' BLAS at start
        try:
            with mp.get_context("spawn").Pool(workers) as pool:
                for arrs in pool.imap(_draw, tasks, chunksize=2):
                    out.append(upload(arrs))
                    if len(out) % 64 == 0:
                        print(json.dumps({"drawing": len(out), "of": len(tasks)}), flush=True)
        finally:
            for k, v in saved.items():
                if v is None:
                    os.environ.pop(k, None)
                else:
                    os.environ[k] = v
        return out

    t0 = time.perf_counter()
    val = draw([10 ** 6 + i for i in range(args.val)])
    pool = draw(range(args.pool)) if args.pool > 0 else None
    print(json.dumps({"drawn": (len(pool) if pool else 0) + len(val), "seconds": round(time.perf_counter() - t0, 1)}),
          flush=True)
    model = NET.PscaNet(args.K, val[0][2], ctx=ctx)
    init = {"from": "schedule rho_0 = 0.5, rho_{k+1} = rho_k (1 - rho_k / 2)"}
    if args.init:
        with open(args.init) as f:
            prev = json.load(f)
        if len(prev["rho"]) != args.K or prev.get("variant") != args.variant:
            raise SystemExit(f"--init {args.init}: K={len(prev['rho'])} {prev.get('variant')}, "
                             f"need K={args.K} {args.variant}")
        with torch.no_grad():
            model.rho.copy_(torch.tensor(prev["rho"], dtype=torch.float32))
        init = {"from": os.path.basename(args.init), "rho": prev["rho"], "train": prev.get("train")}
    opt = torch.optim.Adam(model.parameters(), lr=args.lr)

    def val_eval():
        """Validation loss (the stopping criterion) and, for the record, the
        pooled equal-error rate of the validation outputs."""
        with torch.no_grad():
            tot, scores, truths = 0.0, [], []
            for Sh, S, prm, alpha, g in val:
                x = model(Sh, S, prm)
                tot += float(NET.bce(x, alpha, g, model.known))
                scores.append((x if model.known else x / g).cpu().numpy())
                truths.append(alpha.cpu().numpy())
            model.status.check()
            eer = metrics.equal_error_point(np.concatenate(scores), np.concatenate(truths))[0]
            return tot / len(val), eer

    loss0, eer0 = val_eval()
    history = [{"step": 0, "val_loss": loss0, "val_eer": eer0}]
    best_val, best_rho, best_step, stale = history[0]["val_loss"], model.rho.detach().clone(), 0, 0
    rng = np.random.default_rng([wid, args.batch, args.pool])
    t0 = time.perf_counter()
    visits, next_index, step = 0, 0, 0
    for step in range(1, args.steps + 1):
        if pool is not None:
            batch = [pool[i] for i in rng.choice(len(pool), size=min(args.batch, len(pool)), replace=False)]
        else:
            batch = draw(range(next_index, next_index + args.batch))
            next_index += args.batch
        visits += len(batch)
        loss = NET.train_step(model, opt, batch)
        if step % args.val_every == 0 or step == args.steps:
            vloss, veer = val_eval()
            history.append({"step": step, "train_loss": loss, "val_loss": vloss, "val_eer": veer,
                            "seconds": round(time.perf_counter() - t0, 2)})
            print(json.dumps(history[-1]), flush=True)
            if history[-1]["val_loss"] < best_val:   # keep the step sizes of the best validation loss
                best_val, best_rho, best_step, stale = history[-1]["val_loss"], model.rho.detach().clone(), step, 0
            else:
                stale += 1
                if args.patience and stale >= args.patience:
                    break
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
           "best_step": best_step, "best_val_loss": best_val, "theta": theta,
           "threshold_on": "alpha~" if model.known else "gamma~/g",
           "train": {"steps": step, "max_steps": args.steps, "batch": args.batch, "lr": args.lr,
                     "pool": args.pool, "instance_visits": visits,
                     "distinct_instances": args.pool if args.pool else next_index, "val": args.val,
                     "val_every": args.val_every, "patience": args.patience,
                     "N": args.N, "L": args.L, "M": args.M, "p": args.p, "eps": args.eps,
                     "seeds": "training: [3, i] for i < distinct_instances; validation: [3, 10^6 + i]"},
           "init": init, "history": history}
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    with open(args.out, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", args.out, "theta", theta, "rho", [round(r, 4) for r in out["rho"]], flush=True)
    ctx.close()


if __name__ == "__main__":
    sys.exit(main())
