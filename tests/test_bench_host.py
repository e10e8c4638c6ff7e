"""Host-side arithmetic of bench.py's report (no GPU): the step roofline adds every
stage's algorithmic work at its own peak and sets it against the measured spans."""
import importlib.util
import math
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _counts(**kw):
    c = {"n_cells": 1000, "n_m2l": 5000, "n_visit": 20000, "p2p_pairs": 10 ** 7, "p2p_evaluated": 6 * 10 ** 6,
         "n_m2l_by_order": [0] * 7}
    c.update(kw)
    return c


STAGES = {"t_upward_ms": 1.0, "t_traverse_ms": 2.0, "t_m2l_ms": 3.0, "t_p2p_ms": 4.0, "t_downward_ms": 0.5}


def test_stage_work_follows_the_counting_rules(bench):
    n, p = 4096, 6
    r = bench.stage_rooflines(_counts(), STAGES, 0.25, 10.0, n, p, False, 1, 0)
    s = r["stages"]
    assert s["build"]["work"] == 250 * n and s["build"]["unit"] == "B"
    assert s["p2p"]["work"] == 38 * 10 ** 7
    assert s["m2l"]["work"] == 2 * math.comb(p + 6, 6) * 5000 == 2 * 924 * 5000
    assert s["traversal"]["work"] == 40 * 20000
    assert s["upward"]["work"] == 2 * math.comb(p + 3, 3) * n + 2 * math.comb(p + 6, 6) * 1000
    assert s["downward"]["work"] == 2 * math.comb(p + 6, 6) * 1000 + 6 * math.comb(p + 2, 3) * n
    # times at peak: FP32 form against the FP32 vector peak, traversal against FP64, build against HBM
    assert s["p2p"]["ms_at_peak"] == pytest.approx(38e7 / 157.3e12 * 1e3)
    assert s["traversal"]["ms_at_peak"] == pytest.approx(8e5 / 78.6e12 * 1e3)
    assert s["build"]["ms_at_peak"] == pytest.approx(250 * n / 8e12 * 1e3)
    assert s["p2p"]["frac"] == pytest.approx(s["p2p"]["ms_at_peak"] / 4.0)
    assert r["ms_at_peak"] == pytest.approx(sum(v["ms_at_peak"] for v in s.values()))
    assert r["frac"] == pytest.approx(r["ms_at_peak"] / 10.0)


def test_learned_counts_each_order_and_fp64_uses_its_peak(bench):
    by_order = [1, 2, 3, 4, 5, 6, 7]  # orders 2..8
    r = bench.stage_rooflines(_counts(n_m2l_by_order=by_order), STAGES, 0.25, 10.0, 100, 4, True, 0, 0)
    want = sum(2 * math.comb(o + 6, 6) * c for o, c in zip(range(2, 9), by_order))
    assert r["stages"]["m2l"]["work"] == want
    # expansions at order 8 under the selector, FP64 peak for the FP64 form
    assert r["stages"]["downward"]["work"] == 2 * math.comb(14, 6) * 1000 + 6 * math.comb(10, 3) * 100
    assert r["stages"]["m2l"]["ms_at_peak"] == pytest.approx(want / 78.6e12 * 1e3)


def test_polynomial_split_counts_thirty_flop_per_pair(bench):
    r = bench.stage_rooflines(_counts(), STAGES, 0.25, 10.0, 10, 4, False, 1, 1)
    assert r["stages"]["p2p"]["work"] == 30 * 10 ** 7


def test_p2p_roofline_counts_listed_pairs(bench):
    wl = {"learned": False, "precision": 1, "theta": 0.42, "n_crit": 32}
    r = bench.p2p_roofline({"p2p_pairs": 10 ** 9, "p2p_evaluated": 6 * 10 ** 8}, 2.0, wl, "none", {"p": 6}, 100, 0)
    assert r["flop_per_launch"] == 38 * 10 ** 9
    assert r["achieved"] == pytest.approx(38e9 / 2e-3 / 1e12)
    assert r["frac"] == pytest.approx(38e9 / 2e-3 / 157.3e12)
    assert r["traffic"] is None  # no counters recorded for this workload


def test_fused_roofline_adds_the_m2l_work(bench):
    wl = {"learned": False, "precision": 1, "theta": 0.4, "n_crit": 48}
    st = {"p2p_pairs": 10 ** 9, "p2p_evaluated": 6 * 10 ** 8, "n_m2l": 10 ** 6}
    r = bench.p2p_roofline(st, 2.0, wl, "none", {"p": 5}, 100, 0, fused=True)
    assert r["m2l_flop_in_launch"] == 2 * 462 * 10 ** 6  # C(11, 6) = 462
    assert r["flop_per_launch"] == 38 * 10 ** 9 + 2 * 462 * 10 ** 6
    assert "persistent" in r["kernel"]


def test_cube_sample_takes_whole_seeded_cubes(bench):
    import numpy as np
    rng = np.random.default_rng(0)
    pos = rng.random((200000, 3))
    tg = bench.cube_sample(pos, 0.01, 5)
    side = 1 << bench.CUBE_LEVEL
    cube = np.ravel_multi_index(np.floor(pos * side).astype(np.int64).T, (side,) * 3)
    chosen = np.unique(cube[tg])
    assert len(chosen) <= round(0.01 * side ** 3)
    assert np.array_equal(np.sort(tg), np.nonzero(np.isin(cube, chosen))[0])  # every particle of those cubes
    assert 0.005 < len(tg) / len(pos) < 0.015
    assert np.array_equal(tg, bench.cube_sample(pos, 0.01, 5))  # seeded
    assert len(bench.cube_sample(pos, 1.0, 5)) == len(pos)


def test_per_level_launches_follow_the_library_choice(bench):
    assert bench.per_level(3, {"n_leaves": 10})
    assert not bench.per_level(1, {"n_leaves": 1 << 23})
    assert bench.per_level(0, {"n_leaves": 1 << 22}) and not bench.per_level(0, {"n_leaves": (1 << 22) - 1})
    wl = {"learned": False, "precision": 1, "theta": 0.5, "n_crit": 32}
    r = bench.p2p_roofline({"p2p_pairs": 10, "p2p_evaluated": 8}, 1.0, wl, "none", {"p": 8}, 10, 0, per_level=True)
    assert "per leaf level" in r["launches"]
