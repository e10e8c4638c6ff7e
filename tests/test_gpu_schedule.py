"""Schedule 2: one persistent kernel whose workgroups pull sink leaves (P2P) and then blocks
of 64 M2L pairs from a device queue (the task pool of Sec. 4 as a GPU work queue).
Schedule 3: P2P launched per leaf level as soon as the traversal has listed that level.

Against the FP64 oracle at the FP32 bar of the other parity tests (median <= 1e-6, p99
<= 2e-5 relative), and against schedule 1 (two kernels on two streams) on the same tree:
the same lists and counts, forces equal up to FP32 summation order.  Also: the
polynomial split, a forest with empty boxes, degenerate trees (one particle, one leaf,
no M2L pairs), graph replays, and the autotuner over parameter sets."""
import numpy as np
import pytest

import oracle
from helpers import rel_err
from paper_2006_14952_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
hf = pytest.importorskip("paper_2006_14952_amd")


def dev(x):
    return torch.tensor(np.ascontiguousarray(x), device="cuda")


def opar(prm):
    return oracle.make_params(box=prm.box, rs=prm.r_s, rcut=prm.r_cut, theta=prm.theta, G=prm.G, p=prm.p,
                              ncrit=prm.n_crit, mac_mode=prm.mac_mode, split=prm.split)


def both_schedules(pos, m, prm):
    """Forces and stats under schedule 1 and schedule 2 on one built tree."""
    t = hf.Tree().build(dev(pos), dev(m), prm)
    out = {}
    for sc in (1, 2):
        q = hf.copy_params(prm, schedule=sc)
        print("case: schedule %d, p=%d, split=%d, n=%d" % (sc, prm.p, prm.split, len(pos)), flush=True)
        a = t.short_range(q).cpu().numpy()
        out[sc] = (a, t.stats())
    t.free()
    return out


def check_against_oracle_and_streams(pos, m, prm):
    r = both_schedules(pos, m, prm)
    ref = oracle.fmm(pos, m, opar(prm))
    (a1, s1), (a2, s2) = r[1], r[2]
    for k in ("n_m2l", "n_p2p", "p2p_pairs", "p2p_evaluated", "n_visit"):
        assert s1[k] == s2[k], k
    assert s2["n_m2l"] == ref.stats["n_m2l"] and s2["n_p2p"] == ref.stats["n_p2p"]
    assert s2["p2p_pairs"] == ref.stats["p2p_pairs"]
    e = rel_err(a2, ref.acc)
    d = rel_err(a2, a1)
    print("p=%d split=%d: schedule 2 vs oracle median %.2e p99 %.2e max %.2e; vs schedule 1 max %.2e" % (
        prm.p, prm.split, np.median(e), np.percentile(e, 99), e.max(), d.max()))
    assert np.median(e) <= 1e-6 and np.percentile(e, 99) <= 2e-5 and e.max() <= 1e-3
    assert d.max() <= 1e-5
    return e


@pytest.mark.parametrize("p", [3, 4, 5, 6, 7, 8])
def test_persistent_matches_oracle_and_two_streams(p):
    """Several hundred sink leaves and M2L lists of many 64-pair blocks, a ragged last block."""
    pos, m = inputs.clustered(20000, 12, inputs.rng_for(501, p))
    prm = hf.params(r_s=0.012, r_cut=0.054, theta=0.5, p=p, n_crit=16, precision=1, schedule=2)
    check_against_oracle_and_streams(pos, m, prm)


@pytest.mark.parametrize("p", [4, 7])
def test_persistent_polynomial_split(p):
    pos, m = inputs.clustered(12000, 6, inputs.rng_for(502, p))
    prm = hf.params(r_s=0.012, r_cut=0.06, theta=0.5, p=p, n_crit=16, precision=1, split=1, schedule=2)
    check_against_oracle_and_streams(pos, m, prm)


def test_persistent_degenerate_trees():
    """One particle (one leaf, no lists), one leaf of many particles (P2P only, no M2L),
    two particles across the periodic boundary, and sizes around one wave."""
    prm = hf.params(r_s=0.02, r_cut=0.09, theta=0.5, p=4, n_crit=8, precision=1, schedule=2)
    t = hf.Tree().build(dev(np.array([[0.3, 0.4, 0.5]])), dev(np.array([1.0])), prm)
    assert np.all(t.short_range(prm).cpu().numpy() == 0.0)
    t.free()
    rng = inputs.rng_for(503)
    pos, m = inputs.clustered(300, 1, rng)
    one_leaf = hf.copy_params(prm, n_crit=100000)
    r = both_schedules(pos, m, one_leaf)
    assert r[2][1]["n_m2l"] == 0 and r[2][1]["n_leaves"] == 1
    # one leaf: the same P2P code in the same order under both schedules
    assert rel_err(r[2][0], r[1][0]).max() <= 1e-6
    # the FP32 form's bar against brute force: coordinates relative to a leaf as large as
    # the box carry ~6e-8 absolute rounding, against pair separations of ~1e-3 in the clump
    bf = oracle.bruteforce(pos, m, opar(one_leaf))
    assert np.percentile(rel_err(r[2][0], bf), 99) <= 1e-3
    two = np.array([[0.99, 0.5, 0.5], [0.02, 0.52, 0.47]])
    wm = np.array([0.25, 0.75])
    t = hf.Tree().build(dev(two), dev(wm), hf.copy_params(prm, n_crit=1))
    got = t.short_range(hf.copy_params(prm, n_crit=1)).cpu().numpy()
    t.free()
    bf = oracle.bruteforce(two, wm, opar(prm))
    np.testing.assert_allclose(got, bf, rtol=1e-5)
    for n in (63, 64, 65, 4097):
        pos, m = inputs.clustered(n, 2, rng)
        check_against_oracle_and_streams(pos, m, hf.copy_params(prm, n_crit=4))


def test_persistent_forest_matches_oracle_per_box():
    """A forest with empty, one- and two-particle boxes: the queue covers every box's leaves
    and M2L pairs in one launch."""
    rng = inputs.rng_for(504)
    sizes = [0, 1, 2] + list(rng.integers(100, 4000, 9))
    rng.shuffle(sizes)
    boxes = [inputs.clustered(int(n), 2, rng) if n > 2 else (rng.random((int(n), 3)), np.full(int(n), 0.5))
             for n in sizes]
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    pos = np.concatenate([b[0] for b in boxes])
    m = np.concatenate([b[1] for b in boxes])
    prm = hf.params(r_s=0.02, r_cut=0.09, theta=0.4, p=5, n_crit=16, precision=1, schedule=2)
    t = hf.Tree().build_batched(dev(pos), dev(m), [prm] * len(boxes), off)
    got = t.short_range(prm).cpu().numpy()
    q1 = hf.copy_params(prm, schedule=1)
    t.build_batched(dev(pos), dev(m), [q1] * len(boxes), off)
    got1 = t.short_range(q1).cpu().numpy()
    t.free()
    assert rel_err(got, got1).max() <= 1e-5
    op = opar(prm)
    for b, (bp, bm) in enumerate(boxes):
        if len(bp) == 0:
            continue
        ref = oracle.fmm(bp, bm, op).acc
        e = rel_err(got[off[b]:off[b + 1]], ref)
        assert np.median(e) <= 1e-6 and np.percentile(e, 99) <= 2e-5, (b, np.median(e), np.percentile(e, 99))


def test_persistent_graph_replays():
    """The recorded evaluation under schedule 2: each replay (with eager work and
    synchronisations between) equals the eager evaluation up to FP32 summation order."""
    pos, m = inputs.clustered(30000, 12, inputs.rng_for(505))
    prm = hf.params(r_s=0.012, r_cut=0.054, theta=0.4, p=5, n_crit=32, precision=1, schedule=2)
    t = hf.Tree().build(dev(pos), dev(m), prm)
    ref = t.short_range(prm).cpu().numpy()
    out = torch.empty((len(pos), 3), dtype=torch.float64, device="cuda")
    s = torch.cuda.Stream()
    for rep in range(4):
        out.fill_(np.nan)
        torch.cuda.synchronize()
        t.short_range_graph(prm, out=out, stream=s)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        np.testing.assert_allclose(got, ref, rtol=2e-5, atol=2e-8 * np.abs(ref).max())
    t.free()


def test_autotune_over_parameter_sets():
    """fmm_autotune_params times every set and returns the index of the fastest; the chosen
    set then evaluates to the oracle's forces."""
    rng = inputs.rng_for(506)
    sizes = list(rng.integers(2000, 20000, 6))
    boxes = [inputs.clustered(int(n), 3, rng) for n in sizes]
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    pos, m = np.concatenate([b[0] for b in boxes]), np.concatenate([b[1] for b in boxes])
    prm = hf.params(r_s=0.012, r_cut=0.054, theta=0.4, p=5, n_crit=32, precision=1)
    cands = hf.kernel_candidates(prm, n_crits=(16, 32))
    assert len(cands) == 10
    best, ms = hf.autotune_params(dev(pos), dev(m), cands, reps=1, offsets=off)
    print("sets (n_crit, schedule, m2l_mfma) -> ms:",
          [((c.n_crit, c.schedule, c.m2l_mfma), round(t, 3)) for c, t in zip(cands, ms)])
    assert 0 <= best < len(cands) and all(t > 0 for t in ms)
    assert ms[best] == min(ms)
    q = cands[best]
    got = hf.short_range_batched(dev(pos), dev(m), [q] * len(boxes), off).cpu().numpy()
    b = int(np.argmax(sizes))
    ref = oracle.fmm(boxes[b][0], boxes[b][1], opar(q)).acc
    e = rel_err(got[off[b]:off[b + 1]], ref)
    assert np.median(e) <= 1e-6 and np.percentile(e, 99) <= 2e-5


@pytest.mark.parametrize("precision", [0, 1])
def test_per_level_p2p_matches_oracle_and_after_traversal(precision):
    """Schedule 3 on a clustered box whose leaves span many levels, and on a forest: the
    same counts as schedule 1 and forces equal up to summation order (FP32) or rounding
    (FP64); against the oracle at the form's bar."""
    pos, m = inputs.clustered(30000, 12, inputs.rng_for(507, precision))
    prm = hf.params(r_s=0.012, r_cut=0.054, theta=0.45, p=5, n_crit=8, precision=precision, schedule=3)
    t = hf.Tree().build(dev(pos), dev(m), prm)
    print("case: schedule 3, precision %d" % precision, flush=True)
    a3 = t.short_range(prm).cpu().numpy()
    s3 = t.stats()
    assert s3["max_level"] >= 6
    a1 = t.short_range(hf.copy_params(prm, schedule=1)).cpu().numpy()
    s1 = t.stats()
    t.free()
    for k in ("n_m2l", "n_p2p", "p2p_pairs", "p2p_evaluated"):
        assert s1[k] == s3[k], k
    assert rel_err(a3, a1).max() <= (1e-5 if precision else 1e-12)
    ref = oracle.fmm(pos, m, opar(prm))
    e = rel_err(a3, ref.acc)
    if precision:
        assert np.median(e) <= 1e-6 and np.percentile(e, 99) <= 2e-5
    else:
        assert e.max() <= 1e-9
    # a forest: every box's leaves of a level in one launch
    rng = inputs.rng_for(508, precision)
    sizes = [0, 1] + list(rng.integers(500, 6000, 6))
    boxes = [inputs.clustered(int(n), 2, rng) if n > 1 else (rng.random((int(n), 3)), np.full(int(n), 0.5))
             for n in sizes]
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    fp, fm = np.concatenate([b[0] for b in boxes]), np.concatenate([b[1] for b in boxes])
    q = hf.params(r_s=0.02, r_cut=0.09, theta=0.4, p=4, n_crit=8, precision=precision, schedule=3)
    got = hf.short_range_batched(dev(fp), dev(fm), [q] * len(boxes), off).cpu().numpy()
    for b, (bp, bm) in enumerate(boxes):
        if len(bp) == 0:
            continue
        e = rel_err(got[off[b]:off[b + 1]], oracle.fmm(bp, bm, opar(q)).acc)
        assert (np.percentile(e, 99) <= 2e-5) if precision else (e.max() <= 1e-9), b
