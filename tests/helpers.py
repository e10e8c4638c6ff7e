"""Shared test helpers (error metrics, list comparison).  No arithmetic of the method."""
import numpy as np


def rel_err(a, ref):
    """|a - ref| / |ref| per particle; particles with |ref| = 0 (nothing inside r_cut) are
    scored against the median force magnitude instead."""
    a = np.asarray(a).reshape(-1, 3)
    ref = np.asarray(ref).reshape(-1, 3)
    nb = np.linalg.norm(ref, axis=1)
    floor = np.median(nb[nb > 0]) if np.any(nb > 0) else 1.0
    return np.linalg.norm(a - ref, axis=1) / np.where(nb > 0, nb, floor)


def as_set(triples):
    t = np.asarray(triples, dtype=np.uint64).reshape(-1, 3)
    if t.shape[0] == 0:
        return t
    order = np.lexsort((t[:, 2], t[:, 1], t[:, 0]))
    return t[order]


def same_lists(a, b):
    a, b = as_set(a), as_set(b)
    return a.shape == b.shape and bool(np.all(a == b))
