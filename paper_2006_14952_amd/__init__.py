"""MI355X-native short-range solver of the hybrid PM-FMM method (arXiv:2006.14952).

Thin Python binding of ``libhfmm.so`` (declared in ``include/hfmm.h``).  This module
only marshals arguments: torch tensors provide device memory and the stream, every
step of the method runs in the library's HIP kernels.  If the library is missing the
calls raise; there is no fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os
import re

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhfmm.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "hfmm.h")
_lib = None

FMM_OK, FMM_ERR_ARG, FMM_ERR_NOMEM, FMM_ERR_HIP, FMM_ERR_NAN, FMM_ERR_STATE = 0, -1, -2, -3, -4, -5
PMAX = 8


class FMMError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (code %d)" % (msg, code))
        self.code = code


class Params(C.Structure):
    _fields_ = [("box", C.c_double), ("r_s", C.c_double), ("r_cut", C.c_double), ("theta", C.c_double),
                ("G", C.c_double), ("p", C.c_int), ("n_crit", C.c_int), ("mac_mode", C.c_int),
                ("precision", C.c_int), ("learned", C.c_int), ("split", C.c_int), ("pm_assign", C.c_int),
                ("m2l_mfma", C.c_int), ("schedule", C.c_int), ("deterministic", C.c_int), ("p2p_chunk", C.c_int)]


class Stats(C.Structure):
    _fields_ = [("n", C.c_int64), ("n_cells", C.c_int64), ("n_leaves", C.c_int64), ("max_level", C.c_int64),
                ("n_m2l", C.c_int64), ("n_p2p", C.c_int64), ("p2p_pairs", C.c_int64), ("n_visit", C.c_int64),
                ("levels_traversed", C.c_int64), ("n_m2l_by_order", C.c_int64 * 7),
                ("p2p_evaluated", C.c_int64),
                ("t_tree_ms", C.c_double), ("t_upward_ms", C.c_double), ("t_traverse_ms", C.c_double),
                ("t_m2l_ms", C.c_double), ("t_p2p_ms", C.c_double), ("t_downward_ms", C.c_double),
                ("t_total_ms", C.c_double), ("t_build_ms", C.c_double), ("t_pm_ms", C.c_double),
                ("reserved_d", C.c_double * 6)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if not k.startswith("reserved")}
        d["n_m2l_by_order"] = list(d["n_m2l_by_order"])
        return d


def exported_names():
    """Function names declared by include/hfmm.h."""
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|void|const char \*)\s*(\w+)\s*\(", txt, re.M)))


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise FMMError(FMM_ERR_STATE, "libhfmm.so is not built; run __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        vp, i64, dp = C.c_void_p, C.c_int64, C.c_void_p
        L.fmm_build_tree.argtypes = [C.POINTER(Params), i64, dp, dp, vp, C.POINTER(vp)]
        L.fmm_short_range_forces.argtypes = [vp, C.POINTER(Params), dp, vp]
        L.fmm_short_range_forces_graph.argtypes = [vp, C.POINTER(Params), dp, vp]
        L.pm_long_range_forces.argtypes = [C.POINTER(Params), C.c_int, i64, dp, dp, dp, vp]
        L.hybrid_forces.argtypes = [C.POINTER(Params), C.c_int, i64, dp, dp, dp, vp]
        L.fmm_hybrid_forces_tree.argtypes = [C.POINTER(vp), C.POINTER(Params), C.c_int, i64, dp, dp, dp, vp]
        L.fmm_short_range_forces_batched.argtypes = [C.POINTER(Params), C.c_int, C.POINTER(i64), dp, dp, dp, vp]
        L.fmm_build_tree_batched.argtypes = [C.POINTER(Params), C.c_int, C.POINTER(i64), dp, dp, vp, C.POINTER(vp)]
        L.fmm_get_stats.argtypes = [vp, C.POINTER(Stats)]
        L.fmm_autotune.argtypes = [C.POINTER(Params), C.c_int, C.POINTER(i64), i64, dp, dp, dp, C.POINTER(C.c_int),
                                   C.c_int, C.c_int, vp, C.POINTER(C.c_int), C.POINTER(C.c_double)]
        L.fmm_autotune_params.argtypes = [C.POINTER(Params), C.c_int, C.c_int, C.POINTER(i64), i64, dp, dp, dp,
                                          C.c_int, vp, C.POINTER(C.c_int), C.POINTER(C.c_double)]
        L.fmm_set_timing.argtypes = [vp, C.c_int]
        L.fmm_copy_interactions.argtypes = [vp, C.c_int, vp, i64, C.POINTER(i64)]
        L.fmm_load_mac_model.argtypes = [C.c_char_p]
        fp = C.c_void_p
        L.fmm_set_mac_model.argtypes = [fp, fp, fp, C.c_double, C.c_int]
        L.fmm_mac_training_data.argtypes = [vp, C.POINTER(Params), C.c_double, dp, C.c_double, C.c_int, fp, fp, fp,
                                            fp, i64, C.POINTER(i64), vp]
        L.fmm_mlp_forward.argtypes = [fp, fp, fp, fp, C.c_int, fp, vp]
        L.fmm_mlp_infer.argtypes = [fp, C.c_int, fp, vp]
        L.fmm_mlp_grad.argtypes = [fp, fp, fp, fp, fp, fp, C.c_int, fp, fp, vp]
        L.fmm_mlp_grad_noalloc.argtypes = [fp, fp, fp, fp, fp, fp, C.c_int, fp, fp, vp]
        L.fmm_mlp_adam.argtypes = [fp, fp, fp, fp, i64, C.c_float, C.c_float, C.c_float, C.c_float, C.c_float, vp]
        L.fmm_set_memory_limit.argtypes = [C.c_uint64]
        L.fmm_get_memory_use.argtypes = [C.POINTER(C.c_uint64)]
        L.fmm_free_tree.argtypes = [vp]
        L.fmm_free_tree.restype = None
        L.fmm_last_error.restype = C.c_char_p
        L.fmm_version.restype = C.c_char_p
        _lib = L
    return _lib


def _check(rc):
    if rc != 0:
        raise FMMError(rc, lib().fmm_last_error().decode())


def params(box=1.0, r_s=0.0390625, r_cut=None, theta=0.5, G=1.0, p=4, n_crit=32, mac_mode=0, precision=0,
           learned=0, split=0, pm_assign=0, m2l_mfma=0, schedule=0, deterministic=0, p2p_chunk=0) -> Params:
    """pm_assign: PM mass assignment, 0/2 CIC, 3 TSC, 4 PCS.  m2l_mfma: FP32 M2L kernel,
    0 library's choice, 1 vector ALUs, 2 matrix cores for same-level pairs.  schedule:
    0 library's choice, 1 P2P and M2L on two streams after the traversal, 2 one persistent
    P2P + M2L kernel, 3 as 1 with P2P launched per leaf level during the traversal.
    deterministic: 1 sums every result in a fixed order (bit-identical repeated runs).
    p2p_chunk: P2P sink tile, 16, 32 or 64 particles (0: the library's choice, 32)."""
    if r_cut is None:
        r_cut = 4.5 * r_s
    return Params(float(box), float(r_s), float(r_cut), float(theta), float(G), int(p), int(n_crit), int(mac_mode),
                  int(precision), int(learned), int(split), int(pm_assign), int(m2l_mfma), int(schedule),
                  int(deterministic), int(p2p_chunk))


def copy_params(prm: Params, **changes) -> Params:
    """A copy of prm with the named fields replaced."""
    q = Params()
    C.pointer(q)[0] = prm
    for k, v in changes.items():
        setattr(q, k, v)
    return q


def _stream(stream):
    import torch
    if stream is None:
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    return C.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def _dev64(x, shape_tail=None):
    import torch
    if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == torch.float64 and x.is_contiguous()):
        raise FMMError(FMM_ERR_ARG, "expected a contiguous float64 CUDA tensor")
    if shape_tail is not None and tuple(x.shape[1:]) != shape_tail:
        raise FMMError(FMM_ERR_ARG, "bad tensor shape %s" % (tuple(x.shape),))
    return C.c_void_p(x.data_ptr())


class Tree:
    """A built octree (device-resident) and the lists of its last evaluation."""

    def __init__(self):
        self._h = C.c_void_p()
        self.n = 0
        self._timing = False

    def build(self, pos, mass, prm: Params, stream=None):
        self.n = int(pos.shape[0])
        if mass.shape[0] != self.n:
            raise FMMError(FMM_ERR_ARG, "pos and mass lengths differ")
        fresh = not self._h
        _check(lib().fmm_build_tree(C.byref(prm), self.n, _dev64(pos, (3,)) if self.n else None,
                                    _dev64(mass) if self.n else None, _stream(stream), C.byref(self._h)))
        if fresh and self._timing:
            _check(lib().fmm_set_timing(self._h, 1))
        return self

    def hybrid(self, pos, mass, prm: Params, mesh, out=None, stream=None):
        """Total acceleration, PM long range + short range (fmm_hybrid_forces_tree); the
        tree is (re)built from pos and mass and holds the statistics of the call."""
        import torch
        self.n = int(pos.shape[0])
        if mass.shape[0] != self.n:
            raise FMMError(FMM_ERR_ARG, "pos and mass lengths differ")
        if out is None:
            out = torch.empty((self.n, 3), dtype=torch.float64, device="cuda")
        fresh = not self._h
        _check(lib().fmm_hybrid_forces_tree(C.byref(self._h), C.byref(prm), int(mesh), self.n,
                                            _dev64(pos, (3,)) if self.n else None, _dev64(mass) if self.n else None,
                                            _dev64(out, (3,)) if self.n else None, _stream(stream)))
        if fresh and self._timing and self._h:
            _check(lib().fmm_set_timing(self._h, 1))
        return out

    def build_batched(self, pos, mass, per_box, offsets, stream=None):
        """Forest over the boxes pos[offsets[b]:offsets[b+1]] (all per_box equal)."""
        self.n = int(pos.shape[0])
        if int(offsets[-1]) != self.n or mass.shape[0] != self.n:
            raise FMMError(FMM_ERR_ARG, "offsets, pos and mass disagree")
        nb = len(per_box)
        arr = (Params * nb)(*per_box)
        off = (C.c_int64 * (nb + 1))(*[int(v) for v in offsets])
        fresh = not self._h
        _check(lib().fmm_build_tree_batched(arr, nb, off, _dev64(pos, (3,)) if self.n else None,
                                            _dev64(mass) if self.n else None, _stream(stream), C.byref(self._h)))
        if fresh and self._timing:
            _check(lib().fmm_set_timing(self._h, 1))
        return self

    def short_range(self, prm: Params, out=None, stream=None):
        import torch
        if out is None:
            out = torch.empty((self.n, 3), dtype=torch.float64, device="cuda")
        _check(lib().fmm_short_range_forces(self._h, C.byref(prm), _dev64(out, (3,)) if self.n else None,
                                            _stream(stream)))
        return out

    def short_range_graph(self, prm: Params, out=None, stream=None):
        """Short range through the recorded HIP graph of this tree (fmm_short_range_forces_graph):
        the first call records, later calls with the same out, params and stream replay."""
        import torch
        if out is None:
            out = torch.empty((self.n, 3), dtype=torch.float64, device="cuda")
        _check(lib().fmm_short_range_forces_graph(self._h, C.byref(prm), _dev64(out, (3,)) if self.n else None,
                                                  _stream(stream)))
        return out

    def set_timing(self, on=True):
        """Per-stage HIP-event timing (applied now, or at the first build)."""
        self._timing = bool(on)
        if self._h:
            _check(lib().fmm_set_timing(self._h, int(on)))

    def stats(self):
        s = Stats()
        _check(lib().fmm_get_stats(self._h, C.byref(s)))
        return s.as_dict()

    def interactions(self, kind):
        """(sink key, source key, image) triples of the last evaluation; kind 'm2l' or 'p2p'."""
        k = 1 if kind == "p2p" else 0
        cnt = C.c_int64()
        _check(lib().fmm_copy_interactions(self._h, k, None, 0, C.byref(cnt)))
        out = np.zeros((cnt.value, 3), np.uint64)
        if cnt.value:
            _check(lib().fmm_copy_interactions(self._h, k, C.c_void_p(out.ctypes.data), cnt.value, C.byref(cnt)))
        return out[: cnt.value]

    def free(self):
        if self._h:
            lib().fmm_free_tree(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def short_range(pos, mass, prm: Params, stream=None):
    t = Tree().build(pos, mass, prm, stream)
    try:
        return t.short_range(prm, stream=stream)
    finally:
        t.free()


def autotune(pos, mass, prm: Params, candidates=(16, 24, 32, 48, 64), reps=2, offsets=None, stream=None):
    """Leaf limit with the fastest build + short-range step on these particles
    (fmm_autotune; a forest of boxes when offsets is given); returns
    (best n_crit, {n_crit: ms per step})."""
    import torch
    n = int(pos.shape[0])
    acc = torch.empty((n, 3), dtype=torch.float64, device=pos.device)
    cand = (C.c_int * len(candidates))(*[int(c) for c in candidates])
    ms = (C.c_double * len(candidates))()
    best = C.c_int()
    nbox, off = 1, None
    if offsets is not None:
        nbox = len(offsets) - 1
        off = (C.c_int64 * (nbox + 1))(*[int(v) for v in offsets])
    _check(lib().fmm_autotune(C.byref(prm), nbox, off, n, _dev64(pos, (3,)), _dev64(mass), _dev64(acc, (3,)), cand,
                              len(candidates), int(reps), _stream(stream), C.byref(best), ms))
    return best.value, {int(c): float(m) for c, m in zip(candidates, ms)}


def autotune_params(pos, mass, cands, reps=2, offsets=None, stream=None):
    """Index of the parameter set in cands (a sequence of Params) with the fastest build +
    short-range step on these particles (fmm_autotune_params), and the mean ms per step
    of each set."""
    import torch
    n = int(pos.shape[0])
    acc = torch.empty((n, 3), dtype=torch.float64, device=pos.device)
    arr = (Params * len(cands))(*cands)
    ms = (C.c_double * len(cands))()
    best = C.c_int()
    nbox, off = 1, None
    if offsets is not None:
        nbox = len(offsets) - 1
        off = (C.c_int64 * (nbox + 1))(*[int(v) for v in offsets])
    _check(lib().fmm_autotune_params(arr, len(cands), nbox, off, n, _dev64(pos, (3,)), _dev64(mass),
                                     _dev64(acc, (3,)), int(reps), _stream(stream), C.byref(best), ms))
    return best.value, [float(m) for m in ms]


def sink_tiles(n_crit, chunks):
    """The P2P sink tiles of ``chunks`` that can differ from the default 32 at leaf limit
    n_crit (a tile acts as 32 when no leaf exceeds min(tile, 32) particles); 0 and 32 stay."""
    return tuple(int(c) for c in chunks if c in (0, 32) or n_crit > min(c, 32))


def kernel_candidates(prm: Params, n_crits=(32, 48), chunks=None):
    """The tile and kernel settings the autotuner may vary for prm: each leaf limit in
    n_crits, crossed with the schedules and (FP32 orders 4..8, plain MAC) the two M2L
    kernels, and with the P2P sink tiles in ``chunks`` (None: prm's own); combinations
    the library does not serve are left out, and so are sink tiles that cannot differ
    from the default 32 at that leaf limit (no leaf exceeds min(tile, 32) particles)."""
    fp32_plain = prm.precision == 1 and not prm.learned
    det = bool(prm.deterministic)
    scheds = (1, 2, 3) if fp32_plain and 3 <= prm.p <= 8 and not det else (1, 3)
    mfmas = (1, 2) if fp32_plain and 4 <= prm.p <= 8 and not det else (prm.m2l_mfma,)
    out = []
    for nc in n_crits:
        tiles = (prm.p2p_chunk,) if chunks is None else sink_tiles(nc, chunks)
        for sc in scheds:
            for mf in mfmas:
                if sc == 2 and mf == 2:
                    continue
                for ch in tiles:
                    if sc == 2 and ch not in (0, 32):  # the persistent kernel has tile 32 only
                        continue
                    out.append(copy_params(prm, n_crit=int(nc), schedule=sc, m2l_mfma=mf, p2p_chunk=int(ch)))
    return out


def pm_long_range(pos, mass, prm: Params, mesh, out=None, stream=None):
    import torch
    n = int(pos.shape[0])
    if out is None:
        out = torch.empty((n, 3), dtype=torch.float64, device="cuda")
    _check(lib().pm_long_range_forces(C.byref(prm), int(mesh), n, _dev64(pos, (3,)), _dev64(mass),
                                      _dev64(out, (3,)), _stream(stream)))
    return out


def hybrid(pos, mass, prm: Params, mesh, out=None, stream=None):
    import torch
    n = int(pos.shape[0])
    if out is None:
        out = torch.empty((n, 3), dtype=torch.float64, device="cuda")
    _check(lib().hybrid_forces(C.byref(prm), int(mesh), n, _dev64(pos, (3,)), _dev64(mass), _dev64(out, (3,)),
                               _stream(stream)))
    return out


def short_range_batched(pos, mass, per_box, offsets, out=None, stream=None):
    import torch
    n = int(pos.shape[0])
    if out is None:
        out = torch.empty((n, 3), dtype=torch.float64, device="cuda")
    nb = len(per_box)
    arr = (Params * nb)(*per_box)
    off = (C.c_int64 * (nb + 1))(*[int(v) for v in offsets])
    _check(lib().fmm_short_range_forces_batched(arr, nb, off, _dev64(pos, (3,)), _dev64(mass), _dev64(out, (3,)),
                                                _stream(stream)))
    return out


def set_memory_limit(nbytes):
    """Bound on the device memory the library's buffers hold (0: none); see fmm_set_memory_limit."""
    _check(lib().fmm_set_memory_limit(int(nbytes)))


def memory_in_use():
    v = C.c_uint64()
    _check(lib().fmm_get_memory_use(C.byref(v)))
    return int(v.value)


def load_mac_model(path):
    _check(lib().fmm_load_mac_model(None if path is None else str(path).encode()))


def version():
    return lib().fmm_version().decode()
