"""FP64 CPU oracle of the truncated Cartesian FMM (arXiv:2006.14952, Secs. 2.1-2.3).

TEST INFRASTRUCTURE ONLY.  The test-suite, the smoke check and the CPU-baseline leg of
the benchmark may import this package; the product path never does.  It shares no code
with the GPU library (``paper_2006_14952_amd``): only the seeded input generators of
``paper_2006_14952_amd.inputs`` feed both.

The arithmetic lives in ``hfmm_oracle.c`` (plain C, double precision, OpenMP over
independent sink cells).  This module only compiles it with gcc and marshals arrays.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hfmm_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liborc.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP, no fast-math, no FP contraction)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
               "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class Params(C.Structure):
    _fields_ = [("box", C.c_double), ("rs", C.c_double), ("rcut", C.c_double), ("theta", C.c_double),
                ("G", C.c_double), ("p", C.c_int), ("ncrit", C.c_int), ("mac_mode", C.c_int), ("split", C.c_int)]


STAT_NAMES = ["ncell", "nleaf", "maxlevel", "n_m2l", "n_p2p", "p2p_pairs", "p2p_incut", "n_prune",
              "n_visit", "n_split_sink", "n_split_src", "n_forceopen"]

_dp = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
_lp = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
_up = np.ctypeslib.ndpointer(np.uint64, flags="C_CONTIGUOUS")
_ip = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        L = C.CDLL(_LIB_PATH)
        L.orc_ncoef.argtypes = [C.c_int]; L.orc_ncoef.restype = C.c_int
        L.orc_multi_indices.argtypes = [C.c_int, _ip]
        for nm in ("orc_prefactors_closed", "orc_prefactors_recur", "orc_prefactors_poly"):
            getattr(L, nm).argtypes = [C.c_int, C.c_double, C.c_double, _dp]
        L.orc_prefactors_newton.argtypes = [C.c_int, C.c_double, _dp]
        L.orc_dtensor.argtypes = [C.c_int, _dp, C.c_double, _dp]
        L.orc_dtensor_split.argtypes = [C.c_int, _dp, C.c_double, C.c_double, C.c_int, _dp]
        L.orc_p2m.argtypes = [C.c_int, C.c_long, _dp, _dp, _dp, _dp]
        L.orc_m2m.argtypes = [C.c_int, _dp, _dp, _dp]
        L.orc_m2l.argtypes = [C.c_int, _dp, _dp, C.c_double, _dp]
        L.orc_l2l.argtypes = [C.c_int, _dp, _dp, _dp]
        L.orc_l2p.argtypes = [C.c_int, _dp, _dp, _dp, _dp]
        L.orc_f1.argtypes = [C.c_double, C.c_double]; L.orc_f1.restype = C.c_double
        L.orc_f1_poly.argtypes = [C.c_double, C.c_double]; L.orc_f1_poly.restype = C.c_double
        L.orc_fmm.argtypes = [C.POINTER(Params), C.c_long, _dp, _dp, C.c_long, C.c_void_p, _dp, C.c_int]
        L.orc_fmm.restype = C.c_void_p
        L.orc_free.argtypes = [C.c_void_p]
        L.orc_stats.argtypes = [C.c_void_p, _lp]
        L.orc_seconds.argtypes = [C.c_void_p]; L.orc_seconds.restype = C.c_double
        L.orc_phase_seconds.argtypes = [C.c_void_p, _dp]
        L.orc_ncell.argtypes = [C.c_void_p]; L.orc_ncell.restype = C.c_int
        L.orc_nlist.argtypes = [C.c_void_p, C.c_int]; L.orc_nlist.restype = C.c_long
        L.orc_copy_list.argtypes = [C.c_void_p, C.c_int, _up]
        L.orc_copy_cells.argtypes = [C.c_void_p, _lp, C.c_void_p]
        L.orc_bruteforce.argtypes = [C.POINTER(Params), C.c_double, C.c_long, _dp, _dp, C.c_long, C.c_void_p,
                                     _dp, C.c_int]
        L.orc_bruteforce.restype = C.c_int
        L.orc_max_threads.restype = C.c_int
        _lib = L
    return _lib


def make_params(box=1.0, rs=0.0390625, rcut=0.17578125, theta=0.5, G=1.0, p=4, ncrit=32, mac_mode=0, split=0):
    """split 0: Gaussian (erfc) split of Sec. 2.2 (r_s); 1: polynomial split (r_cut alone)."""
    return Params(float(box), float(rs), float(rcut), float(theta), float(G), int(p), int(ncrit), int(mac_mode),
                  int(split))


def ncoef(p):
    return lib().orc_ncoef(int(p))


def multi_indices(p):
    out = np.zeros((ncoef(p), 3), np.int32)
    lib().orc_multi_indices(int(p), out)
    return out


def prefactors(p, r, rs, method="recur", rc=None):
    """f_(0..p)(r) of Sec. 2.2; method: 'recur' (corrected recurrence), 'closed'
    (general closed form), 'newton' (Eq. (4), rs ignored), 'poly' (polynomial split with
    cutoff rc, rs ignored)."""
    f = np.zeros(p + 1)
    if method == "poly":
        lib().orc_prefactors_poly(int(p), float(r), float(rc), f)
    elif method == "recur":
        lib().orc_prefactors_recur(int(p), float(r), float(rs), f)
    elif method == "closed":
        lib().orc_prefactors_closed(int(p), float(r), float(rs), f)
    else:
        lib().orc_prefactors_newton(int(p), float(r), f)
    return f


def dtensor(p, R, rs, split=0, rc=0.0):
    """D_n(R) for |n| <= p; rs <= 0 gives the Newtonian kernel, split 1 the polynomial split."""
    D = np.zeros(ncoef(p))
    lib().orc_dtensor_split(int(p), np.ascontiguousarray(R, np.float64), float(rs), float(rc), int(split), D)
    return D


def p2m(p, x, m, z):
    M = np.zeros(ncoef(p))
    x = np.ascontiguousarray(x, np.float64).reshape(-1, 3)
    lib().orc_p2m(int(p), x.shape[0], x, np.ascontiguousarray(m, np.float64), np.ascontiguousarray(z, np.float64), M)
    return M


def m2m(p, M, x):
    out = np.zeros(ncoef(p))
    lib().orc_m2m(int(p), np.ascontiguousarray(M, np.float64), np.ascontiguousarray(x, np.float64), out)
    return out


def m2l(p, M, R, rs):
    out = np.zeros(ncoef(p))
    lib().orc_m2l(int(p), np.ascontiguousarray(M, np.float64), np.ascontiguousarray(R, np.float64), float(rs), out)
    return out


def l2l(p, L, x):
    out = np.zeros(ncoef(p))
    lib().orc_l2l(int(p), np.ascontiguousarray(L, np.float64), np.ascontiguousarray(x, np.float64), out)
    return out


def l2p(p, L, y):
    pot = np.zeros(1)
    g = np.zeros(3)
    lib().orc_l2p(int(p), np.ascontiguousarray(L, np.float64), np.ascontiguousarray(y, np.float64), pot, g)
    return pot[0], g


def f1(r, rs):
    return lib().orc_f1(float(r), float(rs))


def f1_poly(r, rc):
    return lib().orc_f1_poly(float(r), float(rc))


class FMMResult:
    """Output of one oracle run: forces plus the tree, interaction lists and counters."""

    def __init__(self, handle, acc):
        self._h = handle
        self.acc = acc
        st = np.zeros(16, np.int64)
        lib().orc_stats(handle, st)
        self.stats = {k: int(st[i]) for i, k in enumerate(STAT_NAMES)}
        self.seconds = lib().orc_seconds(handle)
        ph = np.zeros(5)
        lib().orc_phase_seconds(handle, ph)
        self.phases = dict(zip(("tree", "traversal", "upward", "m2l", "downward_p2p"), ph.tolist()))

    def lists(self, kind):
        """kind 'm2l' or 'p2p': array (n, 3) of (sink key, source key, image)."""
        k = 1 if kind == "p2p" else 0
        n = lib().orc_nlist(self._h, k)
        out = np.zeros((n, 3), np.uint64)
        if n:
            lib().orc_copy_list(self._h, k, out)
        return out

    def cells(self):
        nc = lib().orc_ncell(self._h)
        out = np.zeros((nc, 5), np.int64)
        lib().orc_copy_cells(self._h, out, None)
        return out

    def __del__(self):
        try:
            if self._h:
                lib().orc_free(self._h)
                self._h = None
        except Exception:
            pass


def fmm(pos, mass, params: Params, targets=None, nthreads=0) -> FMMResult:
    """Truncated FMM forces (acceleration, input order).  With ``targets`` only those
    particles get forces (others are 0) and only their sink cells are traversed."""
    pos = np.ascontiguousarray(pos, np.float64).reshape(-1, 3)
    mass = np.ascontiguousarray(mass, np.float64)
    n = pos.shape[0]
    acc = np.zeros((n, 3))
    tg = None
    nt = n
    if targets is not None:
        tg = np.ascontiguousarray(targets, np.int64)
        nt = tg.shape[0]
    h = lib().orc_fmm(C.byref(params), n, pos, mass, nt, tg.ctypes.data if tg is not None else None, acc,
                      int(nthreads))
    if not h:
        raise ValueError("oracle rejected the parameters")
    return FMMResult(h, acc)


def bruteforce(pos, mass, params: Params, targets=None, rc=None, nthreads=0):
    """Hard-cut minimum-image sum over all pairs with 0 < r < rc (default params.rcut)."""
    pos = np.ascontiguousarray(pos, np.float64).reshape(-1, 3)
    mass = np.ascontiguousarray(mass, np.float64)
    n = pos.shape[0]
    tg = None if targets is None else np.ascontiguousarray(targets, np.int64)
    nt = n if tg is None else tg.shape[0]
    out = np.zeros((nt, 3))
    rc = params.rcut if rc is None else rc
    rcode = lib().orc_bruteforce(C.byref(params), float(rc), n, pos, mass, nt,
                                 tg.ctypes.data if tg is not None else None, out, int(nthreads))
    if rcode != 0:
        raise ValueError("bad cutoff for brute force")
    return out


def max_threads():
    return lib().orc_max_threads()
