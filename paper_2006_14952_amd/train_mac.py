"""Train the learned acceptance / order selector on clustered boxes and write the model.

    python -m paper_2006_14952_amd.train_mac [--out FILE] [--n N] [--boxes K] [--epochs E]

Training boxes follow the clustered workload's recipe (50% uniform background, 50% in
Hernquist clumps, r_s = 1.25/128, r_cut = 4.5 r_s) at a reduced N with proportionally
fewer clumps, each with its own seed.  Labels are the smallest expansion order whose
error, measured by the library, is within eps of the particles' total force.  The safety
margin (orders added to the predicted one) is the smallest whose forces on a held-out box
stay within --target of the library's FP64 reference at the 99th percentile.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=None)
    ap.add_argument("--n", type=int, default=262144)
    ap.add_argument("--boxes", type=int, default=3)
    ap.add_argument("--epochs", type=int, default=40)
    ap.add_argument("--theta-max", type=float, default=0.55)
    ap.add_argument("--eps", type=float, default=5e-5)
    ap.add_argument("--stride", type=int, default=1)
    ap.add_argument("--n-crit", type=int, default=32)
    ap.add_argument("--target", type=float, default=5e-4,
                    help="p99 force error, against the library's FP64 reference, that picks the safety margin")
    ap.add_argument("--reselect", default=None,
                    help="only choose the safety margin of an existing model file again (rewritten in place)")
    args = ap.parse_args(argv)

    import torch

    import paper_2006_14952_amd as hf
    from paper_2006_14952_amd import inputs, learned

    pr = inputs.split_params("clustered")
    prm = hf.params(r_s=pr["rs"], r_cut=pr["rcut"], theta=0.3, p=8, n_crit=args.n_crit, precision=1)

    def held_out_safety(params, mu, isd, theta_max):
        # a box of the training recipe with a seed the training boxes do not use
        nclump = max(1, int(round(2000 * args.n / 2 ** 21)))
        pos, m = inputs.clustered(args.n, nclump, inputs.rng_for(901, 0))
        return learned.select_safety(torch.tensor(pos, device="cuda"), torch.tensor(m, device="cuda"), prm, params, mu,
                                     isd, theta_max, target=args.target)

    if args.reselect:
        h = learned.read_model(args.reselect)
        safety, p99 = held_out_safety(h["params"], h["mu"], h["isd"], h["theta_max"])
        cfg = dict(h["config"], safety=safety, safety_p99=p99, target=args.target)
        model = dict(params=h["params"], mu=h["mu"], isd=h["isd"], adam_m=h["adam_m"], adam_v=h["adam_v"],
                     step=h["step"])
        learned.save_model(args.reselect, model, h["theta_max"], h["eps"], safety, cfg)
        print(json.dumps({"rewritten": args.reselect, "safety": safety, "p99": p99}), flush=True)
        return 0
    feats, labels = [], []
    t0 = time.time()
    for b in range(args.boxes):
        rng = inputs.rng_for(900, b)
        nclump = max(1, int(round(2000 * args.n / 2 ** 21)))
        pos, m = inputs.clustered(args.n, nclump, rng)
        d = learned.training_data(torch.tensor(pos, device="cuda"), torch.tensor(m, device="cuda"), prm,
                                  theta_max=args.theta_max, eps=args.eps, stride=args.stride)
        feats.append(d["feats"])
        labels.append(d["labels"])
        print(json.dumps({"box": b, "candidates": int(d["labels"].shape[0]),
                          "class_counts": np.bincount(d["labels"].cpu().numpy(), minlength=8).tolist(),
                          "t": round(time.time() - t0, 1)}), flush=True)
    X = torch.cat(feats).contiguous()
    y = torch.cat(labels).contiguous()
    model = learned.train(X, y, epochs=args.epochs, log=lambda h: print(json.dumps(h), flush=True))
    safety, p99 = held_out_safety(model["params"], model["mu"], model["isd"], args.theta_max)
    cfg = dict(n=args.n, boxes=args.boxes, epochs=args.epochs, theta_max=args.theta_max, eps=args.eps,
               stride=args.stride, n_crit=args.n_crit, r_s=pr["rs"], r_cut=pr["rcut"], samples=int(X.shape[0]),
               safety=safety, safety_p99=p99, target=args.target, final=model["history"][-1])
    out = args.out or learned.DEFAULT_MODEL
    learned.save_model(out, model, args.theta_max, args.eps, safety, cfg)
    print(json.dumps({"written": out, "safety": safety, "t": round(time.time() - t0, 1)}), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
