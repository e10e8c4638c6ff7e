"""CPU checks of the C-ABI library: it loads, exports every declared symbol, and the
binding refuses bad input before touching a GPU."""
import ctypes as C

import pytest

import paper_2006_14952_amd as hf


def test_library_exports_every_declared_symbol():
    names = hf.exported_names()
    assert {"fmm_build_tree", "fmm_short_range_forces", "pm_long_range_forces", "hybrid_forces"} <= set(names)
    L = C.CDLL(hf.LIB_PATH)
    for nm in names:
        assert hasattr(L, nm), nm


def test_param_struct_layout_matches_header():
    assert C.sizeof(hf.Params) == 5 * 8 + 12 * 4  # eleven ints, padded to 8 bytes
    assert C.sizeof(hf.Stats) == 16 * 8 + 16 * 8


def test_version_and_error_string():
    assert "gfx950" in hf.version()
    assert isinstance(hf.lib().fmm_last_error(), bytes)


@pytest.mark.parametrize("bad", [dict(theta=0.0), dict(p=9), dict(p=-1), dict(n_crit=0), dict(r_cut=0.6),
                                 dict(r_s=-1.0), dict(precision=2), dict(mac_mode=8), dict(box=0.0),
                                 dict(schedule=4), dict(schedule=-1), dict(schedule=2),
                                 dict(schedule=2, precision=1, p=2), dict(schedule=2, precision=1, m2l_mfma=2),
                                 dict(schedule=2, precision=1, learned=1),
                                 dict(schedule=2, precision=1, r_cut=0.24)])
def test_bad_params_rejected_without_gpu(bad):
    kw = dict(box=1.0, r_s=0.04, theta=0.5, p=4, n_crit=32)
    kw.update(bad)
    prm = hf.params(**kw)
    h = C.c_void_p()
    rc = hf.lib().fmm_build_tree(C.byref(prm), 0, None, None, None, C.byref(h))
    assert rc == hf.FMM_ERR_ARG
    assert hf.lib().fmm_last_error()


def test_autotune_and_hybrid_tree_reject_bad_arguments_without_gpu():
    L = hf.lib()
    prm = hf.params(box=1.0, r_s=0.04, theta=0.5, p=4, n_crit=32)
    best = C.c_int()
    cand = (C.c_int * 2)(16, 32)
    # no particles / no pointers / no candidates
    assert L.fmm_autotune(C.byref(prm), 1, None, 0, None, None, None, cand, 2, 1, None, C.byref(best), None) == \
        hf.FMM_ERR_ARG
    fake = C.c_void_p(16)  # never dereferenced: the arguments are refused first
    assert L.fmm_autotune(C.byref(prm), 1, None, 10, fake, fake, fake, cand, 0, 1, None, C.byref(best), None) == \
        hf.FMM_ERR_ARG
    bad = (C.c_int * 2)(16, 0)
    assert L.fmm_autotune(C.byref(prm), 1, None, 10, fake, fake, fake, bad, 2, 1, None, C.byref(best), None) == \
        hf.FMM_ERR_ARG
    off = (C.c_int64 * 3)(0, 4, 9)  # offsets[nbox] != n
    assert L.fmm_autotune(C.byref(prm), 2, off, 10, fake, fake, fake, cand, 2, 1, None, C.byref(best), None) == \
        hf.FMM_ERR_ARG
    assert L.fmm_hybrid_forces_tree(None, C.byref(prm), 32, 10, fake, fake, fake, None) == hf.FMM_ERR_ARG
    h = C.c_void_p()
    assert L.fmm_hybrid_forces_tree(C.byref(h), C.byref(prm), 32, 10, None, None, None, None) == hf.FMM_ERR_ARG
    prm.theta = 0.0
    assert L.fmm_hybrid_forces_tree(C.byref(h), C.byref(prm), 32, 10, fake, fake, fake, None) == hf.FMM_ERR_ARG
    # the recorded evaluation refuses a missing tree and bad parameters before any GPU call
    prm.theta = 0.5
    assert L.fmm_short_range_forces_graph(None, C.byref(prm), fake, fake) == hf.FMM_ERR_ARG
    prm.theta = 0.0
    assert L.fmm_short_range_forces_graph(fake, C.byref(prm), fake, fake) == hf.FMM_ERR_ARG


def test_deterministic_field_validated():
    """deterministic is 0 or 1, and refuses the kernels that combine sums with atomics in
    an order of their own (the persistent P2P + M2L kernel, the matrix-core M2L)."""
    L = hf.lib()
    h = C.c_void_p()
    for kw in (dict(deterministic=2), dict(deterministic=-1), dict(deterministic=1, precision=1, p=5, schedule=2),
               dict(deterministic=1, precision=1, p=6, m2l_mfma=2)):
        prm = hf.params(box=1.0, r_s=0.04, theta=0.5, n_crit=32, **{"p": 4, **kw})
        assert L.fmm_build_tree(C.byref(prm), 0, None, None, None, C.byref(h)) == hf.FMM_ERR_ARG, kw
        assert b"deterministic" in L.fmm_last_error(), kw
    # accepted sets pass validation (checked before the particle arguments: n = 0 then fails
    # on the arguments alone, with no GPU call)
    best = C.c_int()
    for kw in (dict(), dict(precision=1, p=6, schedule=3), dict(precision=1, p=8, m2l_mfma=1)):
        prm = hf.params(box=1.0, r_s=0.04, theta=0.5, n_crit=32, deterministic=1, **{"p": 4, **kw})
        arr = (hf.Params * 1)(prm)
        assert L.fmm_autotune_params(arr, 1, 1, None, 0, None, None, None, 1, None, C.byref(best), None) == \
            hf.FMM_ERR_ARG
        assert L.fmm_last_error() == b"bad arguments", kw
    # the autotuner's candidate sets keep to the deterministic kernels
    cands = hf.kernel_candidates(hf.params(p=6, precision=1, deterministic=1), n_crits=(32,))
    assert {(c.schedule, c.m2l_mfma) for c in cands} == {(1, 0), (3, 0)}


def test_persistent_schedule_accepted_where_it_applies():
    """Schedule 2 passes validation for the FP32 plain forms it serves: the parameter sets
    are checked before the particle arguments, so n = 0 fails on the arguments alone."""
    L = hf.lib()
    best = C.c_int()
    for kw in (dict(p=3), dict(p=5), dict(p=8), dict(p=6, split=1, r_cut=0.2), dict(p=4, m2l_mfma=1)):
        prm = hf.params(box=1.0, r_s=0.04, theta=0.5, n_crit=32, precision=1, schedule=2, **kw)
        arr = (hf.Params * 1)(prm)
        assert L.fmm_autotune_params(arr, 1, 1, None, 0, None, None, None, 1, None, C.byref(best), None) == \
            hf.FMM_ERR_ARG
        assert L.fmm_last_error() == b"bad arguments", kw


def test_autotune_params_rejects_bad_arguments_without_gpu():
    L = hf.lib()
    good = hf.params(box=1.0, r_s=0.04, theta=0.5, p=4, n_crit=32)
    bad = hf.params(box=1.0, r_s=0.04, theta=0.5, p=4, n_crit=32, schedule=2)  # FP64: no persistent form
    arr = (hf.Params * 2)(good, bad)
    best = C.c_int()
    fake = C.c_void_p(16)  # never dereferenced: the arguments are refused first
    assert L.fmm_autotune_params(arr, 2, 1, None, 10, fake, fake, fake, 1, None, C.byref(best), None) == \
        hf.FMM_ERR_ARG
    assert b"schedule" in L.fmm_last_error()
    assert L.fmm_autotune_params(arr, 0, 1, None, 10, fake, fake, fake, 1, None, C.byref(best), None) == \
        hf.FMM_ERR_ARG
    assert L.fmm_autotune_params(arr, 1, 1, None, 0, fake, fake, fake, 1, None, C.byref(best), None) == \
        hf.FMM_ERR_ARG


def test_kernel_candidates_cover_the_served_combinations():
    fp32 = hf.params(r_s=0.005, r_cut=0.025, theta=0.4, p=5, precision=1)
    c = hf.kernel_candidates(fp32, n_crits=(32, 48))
    combos = {(q.n_crit, q.schedule, q.m2l_mfma) for q in c}
    assert combos == {(nc, s, m) for nc in (32, 48) for s, m in ((1, 1), (1, 2), (2, 1), (3, 1), (3, 2))}
    assert all(q.p == 5 and q.theta == 0.4 and q.precision == 1 for q in c)
    fp64 = hf.params(r_s=0.005, r_cut=0.025, theta=0.4, p=5, precision=0)
    assert {(q.schedule, q.m2l_mfma) for q in hf.kernel_candidates(fp64)} == {(1, 0), (3, 0)}
    assert {q.p2p_chunk for q in c} == {0}


def test_sink_tile_candidates_skip_tiles_equal_to_the_default():
    """A P2P sink tile is a candidate only where the leaf limit lets it differ from 32:
    16 once leaves may exceed 16 particles, 64 once they may exceed 32."""
    prm = hf.params(r_s=0.005, r_cut=0.025, theta=0.4, p=5, precision=1, schedule=1, m2l_mfma=1)
    got = {(q.n_crit, q.p2p_chunk) for q in hf.kernel_candidates(prm, n_crits=(16, 32, 48, 96), chunks=(16, 32, 64))
           if q.schedule == 1 and q.m2l_mfma == 1}
    assert got == {(16, 32), (32, 16), (32, 32), (48, 16), (48, 32), (48, 64), (96, 16), (96, 32), (96, 64)}


@pytest.mark.parametrize("chunk,schedule", [(8, 0), (24, 0), (128, 0), (-32, 0), (16, 2), (64, 2)])
def test_bad_sink_tile_rejected_without_gpu(chunk, schedule):
    prm = hf.params(box=1.0, r_s=0.04, theta=0.5, p=4, n_crit=32, precision=1, p2p_chunk=chunk, schedule=schedule)
    h = C.c_void_p()
    assert hf.lib().fmm_build_tree(C.byref(prm), 0, None, None, None, C.byref(h)) == hf.FMM_ERR_ARG
    assert b"p2p_chunk" in hf.lib().fmm_last_error() or b"sink tile" in hf.lib().fmm_last_error()
    if schedule == 2:
        cands = hf.kernel_candidates(hf.params(r_s=0.005, r_cut=0.025, p=5, precision=1), n_crits=(96,),
                                     chunks=(16, 32, 64))
        assert all(q.p2p_chunk in (0, 32) for q in cands if q.schedule == 2)


def test_memory_limit_entry_points_on_the_host():
    """Setting the bound and reading the use are host-side (no GPU call); a NULL output is
    an argument error."""
    L = hf.lib()
    assert L.fmm_get_memory_use(None) == hf.FMM_ERR_ARG
    assert L.fmm_set_memory_limit(0) == 0
    assert hf.memory_in_use() >= 0
