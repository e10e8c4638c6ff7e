"""Benchmark: short-range particles/s of the truncated FMM on one MI355X.

A step is one short-range evaluation of a box: octree build (fmm_build_tree) plus
fmm_short_range_forces (upward pass, traversal, M2L, P2P, downward pass), so
particles/s = N / (t_build + t_short).  Inputs are resident in HBM before the timed
region.  Each step is timed with HIP events on the caller's stream (the library's second
stream joins it before the step ends); the line reports the median step.  The PM long
range and the whole hybrid step (build + PM + short range) are timed separately, as is
the plain fixed-order form on the same box when the timed form is the learned selector.
Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload full|large|clustered|batched|uniform]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "short-range particles/s at p99 rel force err ≤1e-3; learned/FP32 vs plain"
PEAK = {"fp32_vector": 157.3e12, "fp64_vector": 78.6e12, "hbm": 8.0e12}
# algorithmic flop per listed P2P pair: the Gaussian split's counting convention (3 sub,
# 3 FMA for r^2, rsqrt, exp, rcp counted 1 each, ~8 erfc approximation, 4 combine, 3 FMA
# accumulate); the polynomial split's factored force law (3 sub, 3 FMA for r^2, rsqrt, 2 mul
# for x = r / r_cut, 1 - x, 3 FMA for the cubic, 4 mul to combine, 1 mul for the mass,
# 3 FMA accumulate)
P2P_FLOP_PER_PAIR = {0: 38.0, 1: 30.0}

# Opening angles: the largest whose p99 error against brute force is <= 1e-3 at the
# configured order.  Clustered (2M, p = 6): theta 0.5 -> 2.7e-3, 0.45 -> 1.9e-3,
# 0.42 -> 9.0e-4 (FP64 oracle on 20000 sampled particles).  Batched (p = 5): theta 0.6 ->
# p99 2.8e-2 .. 4.2e-2 on sampled boxes, 0.4 -> 6.6e-4 .. 9.6e-4.  Large and full (p = 8):
# theta 0.5 meets the bar.  The full box (134M) is timed with the learned selector, the
# plain order-8 form on the same box beside it.
# cpu_cubes: the oracle's sample for cpu_baseline, a seeded fraction of the level-6 cubes
# of the box (all particles in them; 1.0 = the whole input); cpu_cubes_1t the same for the
# one-thread figure.
# n_crit: the leaf limit used without autotuning; tune: the leaf limits the library's
# autotuner chooses from before timing (the default); kernels: the batched line also tunes
# the schedule and the M2L kernel.
WORKLOADS = {
    "full": dict(theta=0.5, precision=1, n_crit=64, tune=(48, 64, 96, 128), learned=True, cpu_cubes=0.0075,
                 cpu_cubes_1t=0.0001),
    "large": dict(theta=0.5, precision=1, n_crit=64, tune=(48, 64, 96), learned=False, cpu_cubes=0.05,
                  cpu_cubes_1t=0.003),
    "clustered": dict(theta=0.42, precision=1, n_crit=48, tune=(32, 48, 64), learned=False, cpu_cubes=0.4,
                      cpu_cubes_1t=0.04),
    "uniform": dict(theta=0.5, precision=0, n_crit=32, tune=(16, 32, 64), learned=False, cpu_cubes=1.0,
                    cpu_cubes_1t=1.0),
    "batched": dict(theta=0.4, precision=1, n_crit=48, tune=(32, 48, 64), kernels=True, learned=False, cpu_cubes=1.0,
                    cpu_cubes_1t=0.15),
}
M2L_KERNELS = {0: "library's choice (vector ALUs)", 1: "vector ALUs", 2: "matrix cores (same-level pairs)"}
TILES = (16, 32, 64)  # P2P sink tiles (particles) the autotuner chooses from
SCHEDULES = {0: "library's choice", 1: "two streams, P2P after the traversal", 2: "one persistent P2P + M2L kernel",
             3: "two streams, P2P per leaf level during the traversal"}
CUBE_LEVEL = 6
CONFIG_SAMPLE_SEED = 777
_T0 = time.perf_counter()


def log(msg):
    """Progress on stderr (the JSON line alone goes to stdout)."""
    print("[bench %6.1fs] %s" % (time.perf_counter() - _T0, msg), file=sys.stderr, flush=True)


def cube_sample(pos, frac, seed):
    """Indices of the particles inside a seeded fraction `frac` of the level-6 cubes of the
    unit box (all of them for frac >= 1): whole cubes, so the oracle's sink leaves inside
    them are complete."""
    if frac >= 1.0:
        return np.arange(len(pos))
    side = 1 << CUBE_LEVEL
    cube = np.ravel_multi_index(np.minimum(np.floor(pos * side), side - 1).astype(np.int64).T, (side,) * 3)
    ncube = max(1, int(round(frac * side ** 3)))
    chosen = np.random.default_rng([2006_14952, seed]).choice(side ** 3, ncube, replace=False)
    return np.nonzero(np.isin(cube, chosen))[0]


def rel_err(got, ref):
    nr = np.linalg.norm(ref, axis=1)
    floor = np.median(nr[nr > 0]) if np.any(nr > 0) else 1.0
    return np.linalg.norm(got - ref, axis=1) / np.where(nr > 0, nr, floor)


def err_stats(e):
    return {"p99": float(np.percentile(e, 99)), "median": float(np.median(e)), "max": float(e.max())}


def p2p_source_sha():
    """Hash of the P2P kernel's sources: stored traffic counters are used only while it holds."""
    h = hashlib.sha256()
    for f in ("p2p.hip",):
        with open(os.path.join(ROOT, "paper_2006_14952_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="full", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", type=int, default=None)
    ap.add_argument("--theta", type=float, default=None)
    ap.add_argument("--n-crit", type=int, default=None)
    ap.add_argument("--autotune", type=int, default=1, choices=(0, 1),
                    help="1 (default): choose n_crit (batched: also schedule and M2L kernel) with the library's "
                         "autotuner before timing; 0: the workload's fixed n_crit (or --n-crit)")
    ap.add_argument("--schedule", type=int, default=0, choices=(0, 1, 2, 3),
                    help="P2P and M2L: 0 library's choice, 1 two kernels on two streams, 2 one persistent kernel, "
                         "3 as 1 with P2P per leaf level during the traversal")
    ap.add_argument("--deterministic", type=int, default=0, choices=(0, 1),
                    help="1: every sum in a fixed order (bit-identical repeated runs; slower M2L)")
    ap.add_argument("--p2p-chunk", type=int, default=0, choices=(0, 16, 32, 64),
                    help="P2P sink tile in particles (0: autotuned with the leaf limit, else fixed)")
    ap.add_argument("--split", type=int, default=0, choices=(0, 1),
                    help="truncation function: 0 Gaussian (erfc) split, 1 polynomial split")
    ap.add_argument("--learned", type=int, default=None, choices=(0, 1),
                    help="1: per-pair acceptance and order from the trained selector (packaged model file)")
    ap.add_argument("--m2l-mfma", type=int, default=0, choices=(0, 1, 2),
                    help="FP32 M2L kernel: 0 library's choice, 1 vector ALUs, 2 matrix cores for same-level pairs")
    ap.add_argument("--plain-steps", type=int, default=3,
                    help="timed steps of the plain fixed-order form beside a learned run (0: skip)")
    ap.add_argument("--pm-steps", type=int, default=2, help="timed hybrid steps (build + PM + short range; 0: skip)")
    ap.add_argument("--cpu", type=int, default=1, choices=(0, 1), help="0: skip the oracle's cpu_baseline")
    ap.add_argument("--accuracy-sample", type=int, default=100000,
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
    for k in ("precision", "theta", "n_crit"):
        if getattr(args, k) is not None:
            wl[k] = getattr(args, k)
    if args.learned is not None:
        wl["learned"] = bool(args.learned)
    cfg = inputs.CONFIGS[args.workload]
    pr = inputs.split_params(args.workload)
    batched = args.workload == "batched"
    log("generating the %s workload" % args.workload)
    t_gen = time.perf_counter()
    if batched:
        sizes = inputs.batched_sizes(cfg["nbox"])
        boxes = [inputs.batched_box(b, sizes[b]) for b in range(len(sizes))]
        offsets = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
        pos_np = np.concatenate([b[0] for b in boxes])
        m_np = np.concatenate([b[1] for b in boxes])
    else:
        pos_np, m_np = inputs.make(args.workload)
    t_gen = time.perf_counter() - t_gen
    n = len(pos_np)
    prm = hf.params(box=1.0, r_s=pr["rs"], r_cut=pr["rcut"], theta=wl["theta"], p=pr["p"], n_crit=wl["n_crit"],
                    precision=wl["precision"], learned=int(wl["learned"]), split=args.split, m2l_mfma=args.m2l_mfma,
                    schedule=args.schedule, deterministic=args.deterministic, p2p_chunk=args.p2p_chunk)
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
    if args.autotune and args.n_crit is None:
        prm, tuned = tune(hf, wl, pos, mass, prm, offsets if batched else None,
                          chunks=TILES if args.p2p_chunk == 0 else (args.p2p_chunk,))
        wl["n_crit"] = prm.n_crit
    acc = torch.empty((n, 3), dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream(dev)
    tree = hf.Tree()
    tree.set_timing(True)

    def step(p_):
        if batched:
            tree.build_batched(pos, mass, [p_] * len(boxes), offsets, stream)
        else:
            tree.build(pos, mass, p_, stream)
        tree.short_range(p_, out=acc, stream=stream)

    def timed(p_, warmup, steps):
        for _ in range(warmup):
            step(p_)
        torch.cuda.synchronize()
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        stats = []
        t0 = time.perf_counter()
        for e0, e1 in evs:
            e0.record(stream)
            step(p_)
            e1.record(stream)
            stats.append(tree.stats())
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / max(steps, 1)
        ms = [e0.elapsed_time(e1) for e0, e1 in evs]
        return ms, wall, stats

    log("inputs ready (%d particles, %.1f s); timing %d steps after %d warm-up" % (n, t_gen, args.steps, args.warmup))
    ms, wall, stats = timed(prm, args.warmup, args.steps)
    log("median step %.2f ms" % float(np.median(ms)))
    st = stats[-1]
    med = float(np.median(ms))
    stage = {k: float(np.median([s[k] for s in stats])) for k in
             ("t_build_ms", "t_upward_ms", "t_traverse_ms", "t_m2l_ms", "t_p2p_ms", "t_downward_ms", "t_total_ms")}
    got = acc.cpu().numpy()

    out = {
        "metric": METRIC,
        "value": n / (med * 1e-3),
        "unit": "particles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": med,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if wl["precision"] else "f64",
        "data": "synthetic",
        "config": {"workload": "%s N=%d (%s), p=%d, theta=%.2f, n_crit=%d, r_s=%.6g, r_cut=%.6g, %s" % (
            args.workload, n, cfg["kind"] + (" %d boxes in one forest" % len(boxes) if batched else ""),
            pr["p"], wl["theta"], wl["n_crit"], pr["rs"], pr["rcut"],
            "FP32 P2P/M2L + FP64 positions/offsets/final sum" if wl["precision"] else "FP64")
            + (", " + sel + " in place of fixed p and theta" if sel else "")
            + (", polynomial split" if args.split else "")
            + "; step = octree build + short-range forces (PM timed separately)",
            "n": n, "p": pr["p"], "theta": wl["theta"], "n_crit": wl["n_crit"], "precision": wl["precision"],
            "split": args.split, "selector": sel or "fixed p and theta", "autotuned_ms": tuned,
            "m2l_kernel": M2L_KERNELS[prm.m2l_mfma], "schedule": SCHEDULES[prm.schedule],
            "p2p_sink_tile": prm.p2p_chunk or 32,
            "sums": "fixed order (deterministic)" if prm.deterministic else "atomics (fastest)"},
        "timing": {"statistic": "median of per-step HIP-event times", "ms_steps": ms,
                   "ms_per_step_mean_wall": wall * 1e3, "input_generation_s": t_gen},
        "roofline": p2p_roofline(st, stage["t_p2p_ms"], wl, args.workload, pr, n, args.split,
                                 fused=prm.schedule == 2, per_level=per_level(prm.schedule, st)),
        "stages_ms": stage,
        "roofline_step": stage_rooflines(st, stage, stage["t_build_ms"], med, n, pr["p"], bool(wl["learned"]),
                                         wl["precision"], args.split),
        "counts": {k: st[k] for k in ("n_cells", "n_leaves", "max_level", "n_m2l", "n_p2p", "p2p_pairs", "n_visit",
                                      "n_m2l_by_order", "p2p_evaluated")},
    }

    # the PM long range and the whole hybrid step (build + PM + short range) on this machine
    if args.pm_steps > 0 and not batched:
        log("hybrid steps (build + PM + short range)")
        hms, pms = [], []
        tree.hybrid(pos, mass, prm, cfg["mesh"], out=acc, stream=stream)
        for _ in range(args.pm_steps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            tree.hybrid(pos, mass, prm, cfg["mesh"], out=acc, stream=stream)
            e1.record(stream)
            torch.cuda.synchronize()
            hms.append(e0.elapsed_time(e1))
            pms.append(tree.stats()["t_pm_ms"])
        out["hybrid"] = {"pm_mesh": cfg["mesh"], "pm_ms": float(np.median(pms)),
                         "hybrid_ms_per_step": float(np.median(hms)),
                         "hybrid_particles_per_s": n / (float(np.median(hms)) * 1e-3)}

    # the plain fixed-order form on the same box (the selector's comparison)
    plain_got = None
    if wl["learned"] and args.plain_steps > 0:
        pp = hf.params(box=1.0, r_s=pr["rs"], r_cut=pr["rcut"], theta=wl["theta"], p=pr["p"], n_crit=wl["n_crit"],
                       precision=wl["precision"], learned=0, split=args.split, m2l_mfma=args.m2l_mfma,
                       schedule=args.schedule, deterministic=args.deterministic, p2p_chunk=args.p2p_chunk)
        log("plain fixed-order form, %d steps" % args.plain_steps)
        pms_, pwall, pstats = timed(pp, 1, args.plain_steps)
        plain_got = acc.cpu().numpy()
        ps = pstats[-1]
        pmed = float(np.median(pms_))
        pstage = {k: float(np.median([s[k] for s in pstats])) for k in stage}
        out["plain"] = {"form": "plain MAC, fixed p=%d, theta=%.2f" % (pr["p"], wl["theta"]),
                        "value": n / (pmed * 1e-3), "ms_per_step": pmed, "ms_steps": pms_, "stages_ms": pstage,
                        "roofline": p2p_roofline(ps, pstage["t_p2p_ms"], wl, args.workload, pr, n, args.split,
                                                 learned=False, per_level=per_level(pp.schedule, ps)),
                        "counts": {k: ps[k] for k in ("n_m2l", "n_p2p", "p2p_pairs", "p2p_evaluated", "n_visit")},
                        "learned_speedup": pmed / med}

    if args.accuracy_sample > 0 or args.cpu:
        import oracle
        if batched:  # the largest box (the oracle runs on one box)
            b = int(np.argmax(sizes))
            bp, bm = boxes[b]
            lo, hi = int(offsets[b]), int(offsets[b + 1])
            got_b, what = got[lo:hi], "the largest box (N=%d)" % len(bp)
            plain_b = None
        else:
            bp, bm, got_b, plain_b, what = pos_np, m_np, got, plain_got, "the box"
        op = oracle.make_params(box=1.0, rs=pr["rs"], rcut=pr["rcut"], theta=wl["theta"], p=pr["p"],
                                ncrit=wl["n_crit"], split=args.split)
        if args.accuracy_sample > 0:
            tg = np.random.default_rng([2006_14952, CONFIG_SAMPLE_SEED]).choice(
                len(bp), min(args.accuracy_sample, len(bp)), replace=False)
            log("brute force on %d particles" % len(tg))
            bf = oracle.bruteforce(bp, bm, op, targets=tg)
            out["accuracy"] = {"sample": "%d seeded random particles of %s" % (len(tg), what),
                               "part": "short range", "reference": "hard-cut brute force (FP64)",
                               "vs_bruteforce": err_stats(rel_err(got_b[tg], bf))}
            if plain_b is not None:
                out["plain"]["vs_bruteforce"] = err_stats(rel_err(plain_b[tg], bf))
        if args.cpu:
            log("oracle cpu_baseline, all threads")
            out["cpu_baseline"], e_or = cpu_baseline(oracle, bp, bm, op, wl["cpu_cubes"], 0, what)
            ref_tg, ref_acc = e_or
            form = plain_b if plain_b is not None else got_b
            out.setdefault("accuracy", {})["vs_oracle"] = dict(
                err_stats(rel_err(form[ref_tg], ref_acc[ref_tg])),
                form="plain p=%d theta=%.2f (the oracle's form)" % (pr["p"], wl["theta"]), sample=len(ref_tg))
            log("oracle cpu_baseline, one thread")
            out["cpu_baseline_1thread"], _ = cpu_baseline(oracle, bp, bm, op, wl["cpu_cubes_1t"], 1, what)
    log("done")
    print(json.dumps(out))
    tree.free()


def cpu_baseline(oracle, pos, m, op, frac, nthreads, what):
    """The FP64 oracle on the particles of a seeded fraction of the level-6 cubes: its tree
    over the whole box, the traversal of the sampled sink cells, the multipoles those
    read, M2L, P2P and the downward pass for the sampled sinks; particles/s = sampled
    particles / wall time."""
    tg = cube_sample(pos, frac, CONFIG_SAMPLE_SEED + nthreads)
    t1 = time.perf_counter()
    res = oracle.fmm(pos, m, op, targets=tg if frac < 1.0 else None, nthreads=nthreads)
    dt = time.perf_counter() - t1
    cores = nthreads if nthreads > 0 else oracle.max_threads()
    rec = {"value": len(tg) / dt, "unit": "particles/s", "cores": cores, "kind": "oracle",
           "sample": ("%d particles in %s of the level-6 cubes of %s (seeded): the tree of the whole box, then "
                      "traversal, multipoles read, M2L, P2P and downward pass for their sink cells; %.1f s"
                      % (len(tg), "all" if frac >= 1.0 else "%.4g%%" % (100 * frac), what, dt)),
           "phases_s": {k: round(v, 3) for k, v in res.phases.items()}}
    if res.stats.get("p2p_pairs"):
        rec["p2p_incut_fraction"] = res.stats["p2p_incut"] / res.stats["p2p_pairs"]
    return rec, (tg, res.acc)


def tune(hf, wl, pos, mass, prm, offsets=None, chunks=None):
    """The workload's launch configuration from the library's autotuner: the leaf limit
    from wl["tune"] crossed with the P2P sink tiles in chunks (and, with wl["kernels"], the
    schedule and the M2L kernel); returns the parameter set and every candidate's ms per step."""
    if wl.get("kernels"):
        log("autotuning n_crit, P2P sink tile, schedule and M2L kernel")
        return tune_kernels(hf, pos, mass, prm, offsets, n_crits=wl["tune"], chunks=chunks)
    log("autotuning n_crit over %s and the P2P sink tile over %s" % (wl["tune"], chunks))
    sets = [hf.copy_params(prm, n_crit=nc, p2p_chunk=ch) for nc in wl["tune"]
            for ch in hf.sink_tiles(nc, chunks or (prm.p2p_chunk,))]
    best, ms = hf.autotune_params(pos, mass, sets, offsets=offsets)
    return sets[best], {"n_crit %d, tile %d" % (c.n_crit, c.p2p_chunk or 32): round(t, 3) for c, t in zip(sets, ms)}


def tune_kernels(hf, pos, mass, prm, offsets=None, n_crits=(32, 48), reps=2, chunks=None):
    """The library's autotuner over the leaf limits n_crits crossed with the P2P sink
    tiles, schedules and M2L kernels that serve prm; returns the fastest parameter set and
    every set's ms."""
    cands = hf.kernel_candidates(prm, n_crits=n_crits, chunks=chunks)
    best, ms = hf.autotune_params(pos, mass, cands, reps=reps, offsets=offsets)
    table = {"n_crit %d, tile %d, %s, M2L on %s" % (c.n_crit, c.p2p_chunk or 32, SCHEDULES[c.schedule],
                                                   M2L_KERNELS[c.m2l_mfma]): round(t, 3)
             for c, t in zip(cands, ms)}
    return cands[best], table


def per_level(schedule, st):
    """Whether the library launched P2P per leaf level beside the traversal (schedule 3, or
    the library's choice for trees of 2^22 leaves or more)."""
    return schedule == 3 or (schedule == 0 and st["n_leaves"] >= (1 << 22))


def p2p_roofline(st, p2p_ms, wl, workload, pr, n, split, learned=None, fused=False, per_level=False):
    """Roofline of the P2P kernel (the dominant one on the clustered boxes): algorithmic
    work = 38 flop per listed pair (30 with the polynomial split) over the launch's
    HIP-event duration on its own stream, against the FP32 (or FP64) vector peak.  Under
    the persistent schedule the kernel is the one P2P + M2L launch and its work adds the
    M2L arithmetic, 2 C(p+6, 6) flop per accepted pair.  With P2P launched per leaf level
    beside the traversal, the duration is the sum of those launches, which share the device
    with the traversal.
    traffic: scaled FETCH_SIZE + WRITE_SIZE of the step's P2P launches from profiles/, when
    those counters were taken on this workload with these parameters, the same launch
    pattern and the current P2P sources."""
    learned = wl["learned"] if learned is None else learned
    flop = P2P_FLOP_PER_PAIR[split] * st["p2p_pairs"]
    m2l_flop = 2 * _binom(pr["p"] + 6, 6) * st["n_m2l"] if fused else 0
    flop += m2l_flop
    peak = PEAK["fp32_vector"] if wl["precision"] else PEAK["fp64_vector"]
    achieved = flop / (p2p_ms * 1e-3) if p2p_ms > 0 else 0.0
    traffic = None
    tf = os.path.join(ROOT, "profiles", "p2p_traffic_%s_fp%d.json" % (workload, 32 if wl["precision"] else 64))
    if os.path.exists(tf) and not fused:
        recs = json.load(open(tf))
        for rec in recs if isinstance(recs, list) else [recs]:
            same = all(rec.get(k) == v for k, v in (("n", n), ("p", pr["p"]), ("theta", wl["theta"]),
                                                    ("n_crit", wl["n_crit"]), ("learned", bool(learned)),
                                                    ("split", split), ("p2p_source_sha", p2p_source_sha()),
                                                    ("per_level", bool(per_level))))
            if same:
                traffic = rec.get("bytes_per_launch")
    return {"kernel": "p2p + m2l (one persistent launch)" if fused else "p2p", "bound": "alu", "achieved": achieved / 1e12, "peak": peak / 1e12, "unit": "TFLOP/s",
            "frac": achieved / peak, "traffic": traffic, "flop_per_launch": flop,
            "unit_of_work": "%.0f flop per listed particle pair" % P2P_FLOP_PER_PAIR[split]
                            + (" + 2 C(p+6,6) flop per M2L pair" if fused else ""),
            "m2l_flop_in_launch": m2l_flop,
            "listed_pairs": st["p2p_pairs"], "evaluated_pairs": st["p2p_evaluated"],
            "p2p_ms_per_launch": p2p_ms,
            "launches": ("one per leaf level, beside the traversal: duration = their sum per step" if per_level
                         else "one per step")}


def _binom(n, k):
    from math import comb
    return comb(n, k)


def stage_rooflines(counts, stages, build_ms, step_ms, n, p, learned, precision, split):
    """Per-stage work at its own peak against the stage's measured span, and the whole step:
    sum of the stages' times at peak / ms per step.  Work per unit: tree 250 B per particle
    (HBM); P2M 2 n_p per particle and M2M, L2L 2 C(p+6,6) per cell; traversal ~40 FP64
    operations per visited pair; M2L 2 C(p+6,6) per accepted pair (at each pair's order for
    the learned selector); P2P 38 flop per listed pair (30 with the polynomial split);
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
        "p2p": (P2P_FLOP_PER_PAIR[split] * counts["p2p_pairs"], "flop", fp, stages["t_p2p_ms"]),
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
