"""The paper's two measurements on synthetic inputs, run through the library.

* ``error_vs_theta``: relative force error of the truncated FMM against opening angle at a
  fixed order (Sec. 2.3, the figure relating error to opening angle at hexadecapole
  order): rms and maximum over all particles.  The reference is the library's own
  evaluation with theta -> 0, where no pair is accepted and every pair inside r_cut is
  summed directly, i.e. the hard-cut short-range sum.
* ``interaction_counts``: numbers of M2L and P2P operations of the truncated MAC against
  a conventional MAC (``mac_mode`` bit 2: item 2 alone), for leaves of at most 1 and 32
  particles (and a coarser leaf limit), in total and per tree level of the sink cell
  (Sec. 3, the uniform case).

Both run for several forms of the MAC (``MAC_MODES``): the library's default (strict item
3, opening size = larger side of the pair), the paper's own size L_B = the source side
with the strict item 3 (mode 2) and with the literal item 3, S_c > r_cut > S_m (mode 3);
and, for the counts, the conventional MAC with either size (modes 4 and 6).

    python -m paper_2006_14952_amd.experiments [--n-clustered 262144] [--thetas 0.2,0.3,...]

prints one JSON document.  Inputs are the seeded generators of ``inputs``; every number
is computed on the GPU by the library.
"""
import argparse
import json

import numpy as np

from . import Tree, inputs, params

_LEVEL_FLOOR = np.array([1 << (3 * l) for l in range(22)], dtype=np.uint64)


def _levels(keys):
    """Tree level of cell keys (1 << 3 level) | morton."""
    return np.searchsorted(_LEVEL_FLOOR, np.asarray(keys, np.uint64), side="right") - 1


def _forces(pos, mass, prm):
    import torch

    t = Tree().build(torch.as_tensor(pos, device="cuda"), torch.as_tensor(mass, device="cuda"), prm)
    acc = t.short_range(prm).cpu().numpy()
    st = t.stats()
    return acc, st, t


# mac_mode values and their names: bit 0 literal item 3, bit 1 source-side size L_B,
# bit 2 conventional MAC (item 2 alone)
MAC_MODES = {0: "truncated, strict item 3, L = larger side (library default)",
             2: "truncated, strict item 3, L = L_B source side (paper's size)",
             3: "truncated, literal item 3, L = L_B (paper's MAC as printed)",
             4: "conventional, L = larger side",
             6: "conventional, L = L_B"}


def error_vs_theta(pos, mass, r_s, r_cut, thetas, p=4, n_crit=32, precision=0, mac_mode=0):
    """rms and max relative force error per theta against the theta -> 0 sum."""
    ref, _, t = _forces(pos, mass, params(r_s=r_s, r_cut=r_cut, theta=1e-3, p=p, n_crit=n_crit))
    t.free()
    nr = np.linalg.norm(ref, axis=1)
    floor = np.median(nr[nr > 0])
    out = []
    for th in thetas:
        acc, st, t = _forces(pos, mass, params(r_s=r_s, r_cut=r_cut, theta=th, p=p, n_crit=n_crit,
                                               precision=precision, mac_mode=mac_mode))
        t.free()
        e = np.linalg.norm(acc - ref, axis=1) / np.where(nr > 0, nr, floor)
        out.append({"theta": th, "rms": float(np.sqrt(np.mean(e * e))), "max": float(e.max()),
                    "p99": float(np.percentile(e, 99)), "n_m2l": st["n_m2l"], "n_p2p": st["n_p2p"]})
    return out


def interaction_counts(pos, mass, r_s, r_cut, theta=0.5, p=4, n_crits=(1, 32), modes=(0, 4)):
    """M2L and P2P counts (cell pairs and listed particle pairs), total and per sink
    level, for each MAC mode (truncated forms against conventional ones)."""
    out = []
    for nc in n_crits:
        for mode in modes:
            _, st, t = _forces(pos, mass, params(r_s=r_s, r_cut=r_cut, theta=theta, p=p, n_crit=nc, mac_mode=mode))
            row = {"n_crit": nc, "mac_mode": mode, "mac": "conventional" if mode & 4 else "truncated",
                   "n_m2l": st["n_m2l"], "n_p2p": st["n_p2p"], "p2p_pairs": st["p2p_pairs"],
                   "n_leaves": st["n_leaves"], "max_level": st["max_level"]}
            for kind in ("m2l", "p2p"):
                lv = _levels(t.interactions(kind)[:, 0])
                row[kind + "_per_level"] = np.bincount(lv, minlength=st["max_level"] + 1).tolist()
            t.free()
            out.append(row)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n-clustered", type=int, default=262144,
                    help="particles of the clustered box for the error sweep (same mix as the 2M workload)")
    ap.add_argument("--thetas", default="0.2,0.3,0.4,0.5,0.6,0.7,0.8")
    args = ap.parse_args()
    res = {}
    # error against opening angle: clustered mix, r_s = 1.25 cells of a 64^3 mesh, p = 4
    n = args.n_clustered
    pos, m = inputs.clustered(n, max(1, round(2000 * n / 2 ** 21)), inputs.rng_for(2006_14952, 91))
    rs = 1.25 / 64
    thetas = [float(x) for x in args.thetas.split(",")]
    res["error_vs_theta"] = {"n": n, "r_s": rs, "r_cut": 4.5 * rs, "p": 4, "mac_modes": MAC_MODES,
                             "rows": {mode: error_vs_theta(pos, m, rs, 4.5 * rs, thetas, mac_mode=mode)
                                      for mode in (0, 2, 3)}}
    # interaction counts: the uniform 32^3 box of the plain workload
    pos, m = inputs.make("uniform")
    pr = inputs.split_params("uniform")
    res["counts_uniform"] = {"n": len(pos), "r_s": pr["rs"], "r_cut": pr["rcut"], "theta": 0.5, "p": 4,
                             "rows": interaction_counts(pos, m, pr["rs"], pr["rcut"], n_crits=(1, 32, 512),
                                                        modes=tuple(MAC_MODES))}
    print(json.dumps(res))


if __name__ == "__main__":
    main()
