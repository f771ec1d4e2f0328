"""Train and evaluate the learned sampling proposal on the GPU.

    python -m paper_2605_29663_amd.train_proposal --samples 50000 --out DIR

Writes DIR/proposal_c2.bin (weights + Adam state), DIR/proposal_c2_eval.json
(held-out cost ratios) and prints progress lines.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--samples", type=int, default=50000)
    ap.add_argument("--parallel", type=int, default=64)
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--eval-states", type=int, default=1000,
                    help="held-out states to evaluate (0: train only)")
    ap.add_argument("--out", default=".")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--max-data-seconds", type=float, default=420.0)
    ap.add_argument("--eval-only", default=None,
                    help="skip data and training: evaluate the weights in this file")
    ap.add_argument("--repeats", type=int, default=4)
    ap.add_argument("--absolute", action="store_true",
                    help="train on absolute sequences instead of residual corrections")
    ap.add_argument("--clutter-keep", type=float, default=None,
                    help="fraction of the corridor clutter kept in training and evaluation "
                         "scenes (default: the module's CLUTTER_KEEP)")
    ap.add_argument("--warm-steps", type=int, default=40,
                    help="closed-loop steps before the first evaluated state of an episode")
    args = ap.parse_args()
    import torch
    import paper_2605_29663_amd as pkg
    from paper_2605_29663_amd import learn

    def log(msg):
        print(msg, flush=True)

    os.makedirs(args.out, exist_ok=True)
    t0 = time.time()
    net = pkg.Proposal(40, 2, hidden=256, max_batch=1024)
    if args.eval_only:
        net.load(args.eval_only)
        n_samples, losses = None, None
        t1 = t2 = time.time()
    else:
        X, U_upd = learn.generate(args.samples, n_parallel=args.parallel, net=net, log=log,
                                  max_seconds=args.max_data_seconds, clutter_keep=args.clutter_keep)
        n_samples = int(X.shape[0])
        log(f"data: {n_samples} samples in {time.time() - t0:.0f} s")
        Y, scale = learn.make_targets(net, X, U_upd, residual=not args.absolute)
        log(f"targets: residual scale {scale:.5f}")
        net.init_params(args.seed)
        t1 = time.time()
        losses = learn.train(net, X, Y, epochs=args.epochs, log=log)
        log(f"train: {time.time() - t1:.0f} s, final loss {losses[-1]:.5f}")
        net.save(os.path.join(args.out, "proposal_c2.bin"))
        t2 = time.time()
    summary = {}
    if args.eval_states > 0:
        costs, fallback = learn.evaluate(net, n_states=args.eval_states, n_parallel=args.parallel,
                                         repeats=args.repeats, log=log, clutter_keep=args.clutter_keep,
                                         warm_steps=args.warm_steps)
        summary = learn.summarize(costs, fallback)
        summary.update(per_state_costs=costs.tolist(), fallback=fallback.tolist())
    summary.update(samples=n_samples, epochs=args.epochs, train_loss=losses, repeats=args.repeats,
                   clutter_keep=learn.CLUTTER_KEEP if args.clutter_keep is None else args.clutter_keep,
                   warm_steps=args.warm_steps,
                   seconds={"data": t1 - t0, "train": t2 - t1, "eval": time.time() - t2})
    name = "proposal_c2_eval.json" if args.eval_states > 0 else "proposal_c2_train.json"
    with open(os.path.join(args.out, name), "w") as f:
        json.dump(summary, f, indent=1)
    log(json.dumps({k: v for k, v in summary.items()
                    if k not in ("train_loss", "per_state_costs", "fallback")}))


if __name__ == "__main__":
    sys.exit(main())
