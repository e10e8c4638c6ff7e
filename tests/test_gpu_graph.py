"""The recorded (HIP graph) short-range evaluation: every replay equals the eager
evaluation of the same tree, with the program's own eager work and synchronisations
between replays; a rebuilt tree is recorded again; a forest of boxes replays as well."""
import numpy as np
import pytest

from paper_2006_14952_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
hf = pytest.importorskip("paper_2006_14952_amd")


def dev(x):
    return torch.tensor(np.ascontiguousarray(x), device="cuda")


def _close(got, ref, rtol):
    # FP32 M2L partial sums are added with atomics in a run-dependent order: rounding level
    np.testing.assert_allclose(got, ref, rtol=rtol, atol=rtol * 1e-3 * np.abs(ref).max())


@pytest.mark.parametrize("precision", [0, 1])
def test_replays_equal_the_eager_evaluation(precision):
    pos, m = inputs.clustered(30000, 12, inputs.rng_for(401, precision))
    prm = hf.params(r_s=0.012, r_cut=0.054, theta=0.4, p=5, n_crit=32, precision=precision)
    rtol = 2e-5 if precision else 1e-11
    print("case: recorded evaluation, precision", precision, flush=True)
    t = hf.Tree().build(dev(pos), dev(m), prm)
    ref = t.short_range(prm).cpu().numpy()
    st_ref = t.stats()
    out = torch.empty((len(pos), 3), dtype=torch.float64, device="cuda")
    s = torch.cuda.Stream()  # a created stream of default priority (the null stream cannot be recorded)
    for rep in range(4):  # first call records, the others replay
        out.fill_(np.nan)  # eager work between replays
        torch.cuda.synchronize()
        t.short_range_graph(prm, out=out, stream=s)
        torch.cuda.synchronize()
        _close(out.cpu().numpy(), ref, rtol)
        st = t.stats()
        assert st["n_m2l"] == st_ref["n_m2l"] and st["n_p2p"] == st_ref["n_p2p"]
        assert st["p2p_pairs"] == st_ref["p2p_pairs"] and st["p2p_evaluated"] == st_ref["p2p_evaluated"]
    # an eager call with other parameters grows buffers the graph uses (order 8 expansions):
    # the next recorded call must record again, and its counts are those of its own evaluation
    prm8 = hf.params(r_s=0.012, r_cut=0.054, theta=0.5, p=8, n_crit=32, precision=precision)
    t.short_range(prm8)
    st8 = t.stats()
    assert st8["n_m2l"] != st_ref["n_m2l"]
    for rep in range(2):
        out.fill_(np.nan)
        torch.cuda.synchronize()
        t.short_range_graph(prm, out=out, stream=s)
        torch.cuda.synchronize()
        _close(out.cpu().numpy(), ref, rtol)
        assert t.stats()["n_m2l"] == st_ref["n_m2l"]
    # a rebuilt tree (other positions) is recorded again
    pos2, m2 = inputs.clustered(24000, 9, inputs.rng_for(402, precision))
    t.build(dev(pos2), dev(m2), prm)
    ref2 = t.short_range(prm).cpu().numpy()
    out2 = torch.empty((len(pos2), 3), dtype=torch.float64, device="cuda")
    for rep in range(3):
        t.short_range_graph(prm, out=out2, stream=s)
        torch.cuda.synchronize()
        _close(out2.cpu().numpy(), ref2, rtol)
    t.free()


def test_forest_replays():
    rng = inputs.rng_for(403)
    sizes = [int(round(2 ** rng.uniform(10, 14))) for _ in range(6)]
    boxes = [inputs.clustered(nb, max(1, nb // 2000), inputs.rng_for(403, b)) for b, nb in enumerate(sizes)]
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    pos = np.concatenate([b[0] for b in boxes])
    m = np.concatenate([b[1] for b in boxes])
    prm = hf.params(r_s=0.02, r_cut=0.09, theta=0.4, p=4, n_crit=16, precision=1)
    print("case: recorded forest of", len(sizes), "boxes", flush=True)
    t = hf.Tree().build_batched(dev(pos), dev(m), [prm] * len(sizes), off)
    ref = t.short_range(prm).cpu().numpy()
    out = torch.empty((len(pos), 3), dtype=torch.float64, device="cuda")
    s = torch.cuda.Stream()
    for rep in range(3):
        out.zero_()
        torch.cuda.synchronize()
        t.short_range_graph(prm, out=out, stream=s)
        torch.cuda.synchronize()
        _close(out.cpu().numpy(), ref, 2e-5)
    with pytest.raises(hf.FMMError):  # the null stream cannot be recorded
        t.short_range_graph(prm, out=out, stream=0)
    t.free()


def test_learned_selector_replays():
    from paper_2006_14952_amd import learned
    learned.load_model()
    pos, m = inputs.clustered(40000, 16, inputs.rng_for(404))
    prm = hf.params(r_s=0.012, r_cut=0.054, theta=0.5, p=8, n_crit=32, precision=1, learned=1)
    print("case: recorded evaluation with the learned selector", flush=True)
    t = hf.Tree().build(dev(pos), dev(m), prm)
    ref = t.short_range(prm).cpu().numpy()
    by_order = t.stats()["n_m2l_by_order"]
    assert sum(by_order) > 0
    out = torch.empty((len(pos), 3), dtype=torch.float64, device="cuda")
    s = torch.cuda.Stream()
    for rep in range(3):
        out.fill_(np.nan)
        torch.cuda.synchronize()
        t.short_range_graph(prm, out=out, stream=s)
        torch.cuda.synchronize()
        _close(out.cpu().numpy(), ref, 2e-5)
        assert t.stats()["n_m2l_by_order"] == by_order
    learned.load_model()  # a model load (same file) makes the next call record again
    t.short_range_graph(prm, out=out, stream=s)
    torch.cuda.synchronize()
    _close(out.cpu().numpy(), ref, 2e-5)
    t.free()


def test_sink_tile_change_records_again_and_forest_tiles_agree():
    """The P2P sink tile is part of the recorded parameters: after replays at tile 32, a call
    with tile 16 records again and its replays equal the eager tile-16 evaluation bit for bit
    (deterministic sums); a forest evaluated at tile 64 equals each box evaluated alone."""
    pos, m = inputs.clustered(30000, 12, inputs.rng_for(403))
    base = hf.params(r_s=0.012, r_cut=0.054, theta=0.45, p=5, n_crit=96, precision=1, deterministic=1, schedule=1)
    t = hf.Tree().build(dev(pos), dev(m), base)
    eager = {c: t.short_range(hf.copy_params(base, p2p_chunk=c)).clone() for c in (32, 16)}
    torch.cuda.synchronize()
    out = torch.empty((len(pos), 3), dtype=torch.float64, device="cuda")
    s = torch.cuda.Stream()
    for c in (32, 32, 16, 16, 16):
        print("case: recorded evaluation, sink tile", c, flush=True)
        out.fill_(np.nan)
        torch.cuda.synchronize()
        t.short_range_graph(hf.copy_params(base, p2p_chunk=c), out=out, stream=s)
        torch.cuda.synchronize()
        assert torch.equal(out, eager[c]), c
    t.free()
    e = np.abs((eager[16] - eager[32]).cpu().numpy()) / np.abs(eager[32].cpu().numpy()).max()
    assert 0 < e.max() < 1e-5  # other FP32 summation groups, same forces
    sizes = [4000, 900, 7000, 1]
    offs = np.concatenate([[0], np.cumsum(sizes)])
    parts = [inputs.clustered(n_b, 4, inputs.rng_for(404, b)) if n_b > 1 else
             (np.array([[0.25, 0.5, 0.75]]), np.array([1.0])) for b, n_b in enumerate(sizes)]
    fpos = np.concatenate([q[0] for q in parts])
    fm = np.concatenate([q[1] / len(q[1]) for q in parts])
    prm = hf.params(r_s=0.02, r_cut=0.09, theta=0.45, p=5, n_crit=96, precision=1, deterministic=1, schedule=1,
                    p2p_chunk=64)
    print("case: forest, sink tile 64", flush=True)
    forest = hf.short_range_batched(dev(fpos), dev(fm), [prm] * len(sizes), offs).cpu().numpy()
    for b in range(len(sizes)):
        alone = hf.short_range(dev(parts[b][0]), dev(parts[b][1] / len(parts[b][1])), prm)
        torch.cuda.synchronize()
        np.testing.assert_allclose(forest[offs[b]:offs[b + 1]], alone.cpu().numpy(), rtol=2e-5,
                                   atol=1e-9 * np.abs(forest).max())
