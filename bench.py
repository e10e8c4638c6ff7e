"""Benchmark: short-range particles/s of the truncated FMM on one MI355X.

A step is one full short-range evaluation of a fresh box: octree build
(fmm_build_tree) plus fmm_short_range_forces (upward pass, traversal, M2L, P2P,
downward pass).  particles/s = N / step time.  Inputs are resident in HBM before the
timed region.  Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload clustered|uniform]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "short-range particles/s at p99 rel force err ≤1e-3; learned/FP32 vs plain"
PEAK = {"fp32_vector": 157.3e12, "fp64_vector": 78.6e12, "hbm": 8.0e12}
# algorithmic flop per evaluated P2P pair: the Gaussian split's counting convention (3 sub,
# 3 FMA for r^2, rsqrt, exp, rcp counted 1 each, ~8 erfc approximation, 4 combine, 3 FMA
# accumulate); the polynomial split's factored force law (3 sub, 3 FMA for r^2, rsqrt, 2 mul
# for x = r / r_cut, 1 - x, 3 FMA for the cubic, 4 mul to combine, 1 mul for the mass,
# 3 FMA accumulate)
P2P_FLOP_PER_PAIR = {0: 38.0, 1: 30.0}

# Opening angles: the largest whose p99 error against brute force is <= 1e-3 at the
# configured order (clustered workload: theta 0.5 -> 2.5e-3, 0.45 -> 1.9e-3, 0.44 and
# 0.42 -> 8.5e-4 (the integer MAC geometry accepts the same pairs), 0.4 -> 2.7e-4).
# Batched: theta 0.6 -> p99 2.8e-2 .. 4.2e-2 on sampled boxes, 0.4 -> 6.6e-4 .. 9.6e-4 at p = 5.
# Large (16.7M clustered, order 8): theta 0.5 meets the bar at p = 8 (p99 7e-4 on the
# clustered mix).  Full (134M, lattice + clumps): the whole hybrid step, PM on a 512^3
# mesh plus the short range, FP32 with the learned selector.
WORKLOADS = {
    "clustered": dict(theta=0.42, precision=1, n_crit=32, learned=False),
    "uniform": dict(theta=0.5, precision=0, n_crit=32, learned=False),
    "batched": dict(theta=0.4, precision=1, n_crit=32, learned=False, autotune=True),
    "large": dict(theta=0.5, precision=1, n_crit=32, learned=False),
    "full": dict(theta=0.5, precision=1, n_crit=32, learned=True, hybrid=True),
}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="clustered", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", type=int, default=None)
    ap.add_argument("--theta", type=float, default=None)
    ap.add_argument("--n-crit", type=int, default=None)
    ap.add_argument("--autotune", type=int, default=None, choices=(0, 1),
                    help="1: choose n_crit with the library's autotuner before timing (default: batched only)")
    ap.add_argument("--split", type=int, default=0, choices=(0, 1),
                    help="truncation function: 0 Gaussian (erfc) split, 1 polynomial split")
    ap.add_argument("--learned", type=int, default=None, choices=(0, 1),
                    help="1: per-pair acceptance and order from the trained selector (packaged model file)")
    ap.add_argument("--cpu-sample", type=int, default=None,
                    help="oracle targets for cpu_baseline (0: skip; default 100000, 0 for large and full)")
    ap.add_argument("--accuracy-sample", type=int, default=20000,
                    help="particles checked against the brute-force sum (0: skip)")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="only run a plain device copy of this many bytes (calibrates HBM counters) and exit")
    args = ap.parse_args()
    if args.copy_bytes:
        copy_calibration(args.copy_bytes)
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path (--gpus %d requested)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2006_14952_amd as hf
    from paper_2006_14952_amd import inputs

    wl = dict(WORKLOADS[args.workload])
    if args.precision is not None:
        wl["precision"] = args.precision
    if args.theta is not None:
        wl["theta"] = args.theta
    if args.n_crit is not None:
        wl["n_crit"] = args.n_crit
    if args.learned is not None:
        wl["learned"] = bool(args.learned)
    hybrid = wl.get("hybrid", False)
    cfg = inputs.CONFIGS[args.workload]
    pr = inputs.split_params(args.workload)
    batched = args.workload == "batched"
    if batched:
        sizes = inputs.batched_sizes(cfg["nbox"])
        boxes = [inputs.batched_box(b, sizes[b]) for b in range(len(sizes))]
        offsets = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
        pos_np = np.concatenate([b[0] for b in boxes])
        m_np = np.concatenate([b[1] for b in boxes])
    else:
        pos_np, m_np = inputs.make(args.workload)
    n = len(pos_np)
    prm = hf.params(box=1.0, r_s=pr["rs"], r_cut=pr["rcut"], theta=wl["theta"], p=pr["p"], n_crit=wl["n_crit"],
                    precision=wl["precision"], learned=int(wl["learned"]), split=args.split)
    sel = None
    if wl["learned"]:
        from paper_2006_14952_amd import learned
        learned.load_model()
        hdr = learned.read_model(learned.DEFAULT_MODEL)
        sel = "learned selector (theta_max %.2f, eps %.0e, safety %d)" % (hdr["theta_max"], hdr["eps"],
                                                                          hdr["safety"])
    dev = torch.device("cuda:0")
    pos = torch.tensor(pos_np, device=dev)
    mass = torch.tensor(m_np, device=dev)
    tuned = None
    if (args.autotune if args.autotune is not None else wl.get("autotune", False)) and not hybrid:
        best, ms = hf.autotune(pos, mass, prm, offsets=offsets if batched else None)
        prm.n_crit = wl["n_crit"] = best
        tuned = {str(k): round(v, 3) for k, v in ms.items()}
    acc = torch.empty((n, 3), dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream(dev)
    tree = hf.Tree()

    mesh = cfg["mesh"]

    def step():
        if hybrid:
            tree.hybrid(pos, mass, prm, mesh, out=acc, stream=stream)
            return
        if batched:
            tree.build_batched(pos, mass, [prm] * len(boxes), offsets, stream)
        else:
            tree.build(pos, mass, prm, stream)
        tree.short_range(prm, out=acc, stream=stream)

    for _ in range(args.warmup):
        step()
    tree.set_timing(True)
    torch.cuda.synchronize()
    p2p_ms, build_ms, pm_ms, stage = [], [], [], {}
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
        s = tree.stats()
        p2p_ms.append(s["t_p2p_ms"])
        build_ms.append(s["t_build_ms"])
        pm_ms.append(s["t_pm_ms"])
        for k in ("t_upward_ms", "t_traverse_ms", "t_m2l_ms", "t_p2p_ms", "t_downward_ms", "t_total_ms"):
            stage.setdefault(k, []).append(s[k])
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    st = tree.stats()

    flop_launch = P2P_FLOP_PER_PAIR[args.split] * st["p2p_evaluated"]  # pairs the kernel evaluates
    p2p_s = float(np.mean(p2p_ms)) * 1e-3
    peak = PEAK["fp32_vector"] if wl["precision"] else PEAK["fp64_vector"]
    achieved = flop_launch / p2p_s
    traffic = None
    tf = os.path.join(ROOT, "profiles", "p2p_traffic_%s_fp%d.json" % (args.workload, 32 if wl["precision"] else 64))
    if os.path.exists(tf):  # counters taken on this workload with the same parameters, else not reported
        rec = json.load(open(tf))
        same = all(rec.get(k, 0 if k == "split" else None) == v
                   for k, v in (("n", n), ("p", pr["p"]), ("theta", wl["theta"]), ("n_crit", wl["n_crit"]),
                                ("learned", bool(wl["learned"])), ("split", args.split)))
        if same:
            traffic = rec.get("bytes_per_launch")

    out = {
        "metric": METRIC,
        "value": n / dt,
        "unit": "particles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if wl["precision"] else "f64",
        "data": "synthetic",
        "config": {"workload": "%s N=%d (%s), p=%d, theta=%.2f, n_crit=%d, r_s=%.6g, r_cut=%.6g, %s" % (
            args.workload, n, cfg["kind"] + (" %d boxes in one forest" % len(boxes) if batched else ""),
            pr["p"], wl["theta"], wl["n_crit"], pr["rs"], pr["rcut"],
            "FP32 P2P/M2L + FP64 positions/offsets/final sum" if wl["precision"] else "FP64")
            + (", " + sel + " in place of p and theta" if sel else "")
            + (", polynomial split" if args.split else "")
            + (", full hybrid step: PM on %d^3 mesh + short range" % mesh if hybrid else ""),
            "n": n, "p": pr["p"], "theta": wl["theta"], "n_crit": wl["n_crit"], "precision": wl["precision"],
            "split": args.split,
            "selector": sel or "fixed p and theta", "autotuned_n_crit_ms": tuned},
        "roofline": {"kernel": "p2p", "bound": "alu", "achieved": achieved / 1e12, "peak": peak / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / peak, "traffic": traffic,
                     "flop_per_launch": flop_launch, "p2p_ms_per_launch": p2p_s * 1e3},
        "stages_ms": {k: float(np.mean(v)) for k, v in stage.items()},
        "roofline_step": stage_rooflines(st, {k: float(np.mean(v)) for k, v in stage.items()}, float(np.mean(build_ms)),
                                         dt * 1e3, n, pr["p"], bool(wl["learned"]), wl["precision"], args.split),
        "build_ms": float(np.mean(build_ms)),
        "pm_ms": float(np.mean(pm_ms)) if hybrid else None,
        "counts": {k: st[k] for k in ("n_cells", "n_leaves", "max_level", "n_m2l", "n_p2p", "p2p_pairs", "n_visit",
                                      "n_m2l_by_order", "p2p_evaluated")},
    }

    cpu_sample = args.cpu_sample if args.cpu_sample is not None else (
        0 if args.workload in ("large", "full") else 100000)
    if cpu_sample > 0 or args.accuracy_sample > 0:
        import oracle
        if batched:  # sampled particles of the largest box (the oracle runs on that box alone)
            b = int(np.argmax(sizes))
            bp, bm = boxes[b]
            got = acc.cpu().numpy()[offsets[b]:offsets[b + 1]]
            what = "random particles of the largest box (N=%d)" % len(bp)
        else:
            bp, bm = pos_np, m_np
            if hybrid:  # the short-range part alone, on the tree of the last step
                got = tree.short_range(prm, stream=stream).cpu().numpy()
            else:
                got = acc.cpu().numpy()
            what = "random particles of the same box"
        tg = inputs.rng_for(CONFIG_SAMPLE_SEED).choice(len(bp), min(max(cpu_sample, args.accuracy_sample), len(bp)),
                                                       replace=False)
        op = oracle.make_params(box=1.0, rs=pr["rs"], rcut=pr["rcut"], theta=wl["theta"], p=pr["p"],
                                ncrit=wl["n_crit"], split=args.split)
        bf = oracle.bruteforce(bp, bm, op, targets=tg)
        ref_norm = np.linalg.norm(bf, axis=1)
        floor = np.median(ref_norm[ref_norm > 0])
        e_bf = np.linalg.norm(got[tg] - bf, axis=1) / np.where(ref_norm > 0, ref_norm, floor)
        out["accuracy"] = {"sample": len(tg), "part": "short range", "p99_vs_bruteforce": float(np.percentile(e_bf, 99)),
                           "median_vs_bruteforce": float(np.median(e_bf)), "max_vs_bruteforce": float(e_bf.max())}
        if cpu_sample > 0:
            tgc = tg[:cpu_sample]
            t1 = time.perf_counter()
            res = oracle.fmm(bp, bm, op, targets=tgc)
            t_or = time.perf_counter() - t1
            e_or = (np.linalg.norm(got[tgc] - res.acc[tgc], axis=1)
                    / np.maximum(np.linalg.norm(res.acc[tgc], axis=1), 1e-300))
            out["cpu_baseline"] = {"value": len(tgc) / t_or, "unit": "particles/s", "cores": oracle.max_threads(),
                                   "kind": "oracle",
                                   "sample": "%d %s: its full tree and upward pass, then traversal/M2L/P2P/downward"
                                             " for their sink cells only; %.1f s" % (len(tgc), what, t_or)}
            # the share of listed P2P pairs that lie inside r_cut, from the oracle's own lists
            # of the sampled sink leaves (the GPU counts listed and evaluated pairs only)
            if res.stats.get("p2p_pairs"):
                out["counts"]["p2p_incut_fraction_sampled"] = res.stats["p2p_incut"] / res.stats["p2p_pairs"]
            out["accuracy"].update({"oracle_form": "plain p=%d theta=%.2f" % (pr["p"], wl["theta"]),
                                    "median_vs_oracle": float(np.median(e_or)),
                                    "p99_vs_oracle": float(np.percentile(e_or, 99)), "max_vs_oracle": float(e_or.max())})
    print(json.dumps(out))
    tree.free()


CONFIG_SAMPLE_SEED = 777


def _binom(n, k):
    from math import comb
    return comb(n, k)


def stage_rooflines(counts, stages, build_ms, step_ms, n, p, learned, precision, split):
    """Per-stage work at its own peak against the stage's measured span, and the whole step:
    sum of the stages' times at peak / ms per step.  Work per unit: tree 250 B per particle
    (HBM); P2M 2 n_p per particle and M2M, L2L 2 C(p+6,6) per cell; traversal ~40 FP64
    operations per visited pair; M2L 2 C(p+6,6) per accepted pair (at each pair's order for
    the learned selector); P2P 38 flop per evaluated pair (30 with the polynomial split);
    L2P 6 C(p+2,3) per particle.  Stages on the two streams overlap, so their spans do too."""
    pe = 8 if learned else p  # expansions are kept at order 8 under the selector
    fp = PEAK["fp32_vector"] if precision else PEAK["fp64_vector"]
    if learned:
        m2l = sum(2 * _binom(o + 6, 6) * c for o, c in zip(range(2, 9), counts["n_m2l_by_order"]))
    else:
        m2l = 2 * _binom(p + 6, 6) * counts["n_m2l"]
    rows = {
        "build": (250.0 * n, "B", PEAK["hbm"], build_ms),
        "upward": (2.0 * _binom(pe + 3, 3) * n + 2.0 * _binom(pe + 6, 6) * counts["n_cells"], "flop", fp,
                   stages["t_upward_ms"]),
        "traversal": (40.0 * counts["n_visit"], "op", PEAK["fp64_vector"], stages["t_traverse_ms"]),
        "m2l": (float(m2l), "flop", fp, stages["t_m2l_ms"]),
        "p2p": (P2P_FLOP_PER_PAIR[split] * counts["p2p_evaluated"], "flop", fp, stages["t_p2p_ms"]),
        "downward": (2.0 * _binom(pe + 6, 6) * counts["n_cells"] + 6.0 * _binom(pe + 2, 3) * n, "flop", fp,
                     stages["t_downward_ms"]),
    }
    out, at_peak = {}, 0.0
    for k, (w, unit, peak, ms) in rows.items():
        t = w / peak * 1e3
        at_peak += t
        out[k] = {"work": w, "unit": unit, "ms_at_peak": t, "ms": ms, "frac": t / ms if ms > 0 else None}
    return {"stages": out, "ms_at_peak": at_peak, "frac": at_peak / step_ms}


def copy_calibration(nbytes):
    """A plain elementwise copy (reads and writes nbytes each) for scaling the FETCH_SIZE
    and WRITE_SIZE counters of the profiled kernels."""
    import torch
    n = nbytes // 4
    x = torch.ones(n, dtype=torch.float32, device="cuda:0")
    y = torch.empty_like(x)
    for _ in range(3):
        torch.mul(x, 1.0, out=y)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n * 4, "copy_bytes_written": n * 4, "launches": 3}))

if __name__ == "__main__":
    main()
