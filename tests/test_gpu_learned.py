"""GPU checks of the learned acceptance / order selector: training kernels against an
FP64 backpropagation reference, BF16 MFMA inference against a
BF16-rounded reference, and the label generator against the oracle's own expansions."""
import os

import numpy as np
import pytest

import oracle
from oracle import mlp as omlp
from paper_2006_14952_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
hf = pytest.importorskip("paper_2006_14952_amd")
from paper_2006_14952_amd import learned  # noqa: E402


def _batch(B, seed):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((B, 16)).astype(np.float32) * 2 + 1
    y = rng.integers(0, 8, B).astype(np.int32)
    w = learned.init_params(seed) + rng.standard_normal(5768).astype(np.float32) * 0.01
    mu = rng.standard_normal(16).astype(np.float32) * 0.3
    isd = (0.5 + rng.random(16)).astype(np.float32)
    cw = (0.5 + rng.random(8)).astype(np.float32)
    return X, y, w, mu, isd, cw


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda")


def test_mlp_gradient_matches_fp64_backprop():
    X, y, w, mu, isd, cw = _batch(300, 1)
    loss, g = learned.grad(_dev(w), _dev(mu), _dev(isd), _dev(X), _dev(y), _dev(cw))
    lref, gref = omlp.loss_and_grad(w.astype(np.float64), X, y, cw, mu, isd)
    assert abs(loss - lref) < 1e-5 * max(1.0, abs(lref))
    g = g.cpu().numpy()
    np.testing.assert_allclose(g, gref, rtol=2e-3, atol=2e-6 * np.abs(gref).max())
    # the reference itself is pinned on the CPU (tests/test_mlp_oracle.py): torch autograd,
    # torch.optim.Adam, torch's bfloat16 rounding and central finite differences


def test_adam_matches_reference():
    rng = np.random.default_rng(3)
    w = rng.standard_normal(5768).astype(np.float32)
    g = rng.standard_normal(5768).astype(np.float32)
    m = rng.standard_normal(5768).astype(np.float32) * 0.1
    v = rng.random(5768).astype(np.float32) * 0.1
    wd, md, vd = _dev(w.copy()), _dev(m.copy()), _dev(v.copy())
    learned.adam(wd, _dev(g), md, vd, 7, 1e-3, wd=1e-4)
    wr, mr, vr = omlp.adam(w.astype(np.float64), g, m, v, 7, 1e-3, 0.9, 0.999, 1e-8, 1e-4)
    np.testing.assert_allclose(wd.cpu().numpy(), wr, rtol=1e-5, atol=1e-6)
    np.testing.assert_allclose(md.cpu().numpy(), mr, rtol=1e-5, atol=1e-7)


def test_forward_fp32_and_bf16_mfma_inference():
    X, y, w, mu, isd, cw = _batch(333, 4)
    Z32 = learned.forward(_dev(w), _dev(mu), _dev(isd), _dev(X)).cpu().numpy()
    Z64 = omlp.forward(w.astype(np.float64), X, mu, isd)[3]
    np.testing.assert_allclose(Z32, Z64, rtol=1e-4, atol=1e-4 * np.abs(Z64).max())
    learned.set_model(w, mu, isd, 0.5, 0)
    try:
        Zb = learned.infer(_dev(X)).cpu().numpy()
    finally:
        learned.unload_model()
    Zr = omlp.forward_bf16(w, X, mu, isd)
    scale = np.abs(Zr).max()
    assert np.abs(Zb - Zr).max() < 2e-2 * scale
    assert np.mean(Zb.argmax(1) == Zr.argmax(1)) > 0.97


def _key_cell(key, box=1.0):
    key = int(key)
    lvl = (key.bit_length() - 1) // 3
    ix = iy = iz = 0
    for b in range(lvl):
        d = (key >> (3 * b)) & 7
        ix |= ((d >> 2) & 1) << b
        iy |= ((d >> 1) & 1) << b
        iz |= (d & 1) << b
    h = box / 2 ** lvl
    return lvl, h, np.array([(ix + 0.5) * h, (iy + 0.5) * h, (iz + 0.5) * h])


def test_labels_match_oracle_expansions():
    pos, m = inputs.clustered(20000, 8, inputs.rng_for(401))
    rs, rc = 0.02, 0.09
    prm = hf.params(r_s=rs, r_cut=rc, theta=0.3, p=8, n_crit=16, precision=1)
    d = learned.training_data(torch.tensor(pos, device="cuda"), torch.tensor(m, device="cuda"), prm,
                              theta_max=0.55, eps=5e-5, stride=3, with_pairs=True)
    errs = d["errs"].cpu().numpy().astype(np.float64)
    labels = d["labels"].cpu().numpy()
    pairs = d["pairs"].cpu().numpy().view(np.uint64)
    feats = d["feats"].cpu().numpy()
    aref = np.linalg.norm(d["aref"].cpu().numpy(), axis=1)
    assert len(labels) > 1000
    res = oracle.fmm(pos, m, oracle.make_params(rs=rs, rcut=rc, theta=0.3, p=8, ncrit=16))
    cells = res.cells()
    orig = np.zeros(len(pos), np.int64)
    oracle.lib().orc_copy_cells(res._h, cells, orig.ctypes.data)
    rng_of = {int(k): (int(b), int(e)) for k, _, b, e, _ in cells}
    x = np.mod(pos, 1.0)
    rng = np.random.default_rng(5)
    checked = 0
    for c in rng.permutation(len(labels)):
        ka, kb, s = (int(v) for v in pairs[c])
        ba, ea = rng_of[ka]
        bb, eb = rng_of[kb]
        if (ea - ba) * (eb - bb) > 3000:
            continue
        ia, ib = orig[ba:ea], orig[bb:eb]
        la, hA, zA = _key_cell(ka)
        lb, hB, zB = _key_cell(kb)
        sh = np.array([s // 9 - 1, (s // 3) % 3 - 1, s % 3 - 1], float)
        R = zA - (zB + sh)
        assert abs(feats[c, 0] - max(hA, hB) / np.linalg.norm(R)) < 1e-5
        assert abs(feats[c, 3] - np.linalg.norm(R) / rs) < 1e-4 * np.linalg.norm(R) / rs
        M = oracle.p2m(8, x[ib] + sh, m[ib], zB + sh)
        direct = np.zeros((len(ia), 3))
        for t, i in enumerate(ia):
            dd = x[i] - (x[ib] + sh)
            r = np.linalg.norm(dd, axis=1)
            ok = (r > 0) & (r < rc)
            direct[t] = (m[ib][ok, None] * np.array([oracle.f1(v, rs) for v in r[ok]])[:, None] * dd[ok]).sum(0)
        for p in range(2, 9):
            L = oracle.m2l(p, M[:oracle.ncoef(p)], R, rs)
            e = max(np.linalg.norm(oracle.l2p(p, L, x[i] - zA)[1] - direct[t]) / aref[i] for t, i in enumerate(ia))
            assert abs(e - errs[c, p - 2]) <= 1e-3 * e + 1e-9, (c, p, e, errs[c, p - 2])
        ok = [p for p in range(2, 9) if errs[c, p - 2] <= 5e-5]
        assert labels[c] == (ok[0] - 1 if ok else 0)
        checked += 1
        if checked >= 25:
            break
    assert checked >= 10


def test_learned_selector_accuracy_and_gain():
    """What the trained selector gains over the method without it, on the 16.7M clustered
    box (a box of the training recipe it was not trained on), against the plain MAC at the
    settings that just meet p99 <= 1e-3 against brute force: order 8 at theta 0.5 and
    order 6 at theta 0.42.  Each form: p99 against brute force on 2000 sampled particles,
    median time of a build + short-range step over 5 timed steps, listed P2P pairs and M2L
    arithmetic (2 C(p+6, 6) flop per pair at the order each pair is evaluated at).

    Asserted: every form meets the bar; the selector needs less M2L arithmetic than plain
    order 8 and fewer listed P2P pairs than plain order 6.  The step times are printed and
    recorded as they are: the selector's step is not faster than the best plain form (its
    network and feature work in the traversal cost more than the M2L and P2P work it
    saves on this machine)."""
    if not os.path.exists(learned.DEFAULT_MODEL):
        pytest.skip("no trained model file")
    from math import comb
    pr = inputs.split_params("large")
    pos, m = inputs.make("large")
    n = len(pos)
    dpos, dm = torch.tensor(pos, device="cuda"), torch.tensor(m, device="cuda")
    tg = inputs.rng_for(402).choice(n, 2000, replace=False)
    op = oracle.make_params(box=1.0, rs=pr["rs"], rcut=pr["rcut"], theta=0.5, p=8, ncrit=32)
    bf = oracle.bruteforce(pos, m, op, targets=tg)
    ref = np.linalg.norm(bf, axis=1)
    learned.load_model()

    def run(**kw):
        prm = hf.params(r_s=pr["rs"], r_cut=pr["rcut"], n_crit=32, precision=1, **kw)
        t = hf.Tree()
        t.set_timing(True)
        ms = []
        for k in range(7):
            t.build(dpos, dm, prm)
            a = t.short_range(prm)
            st = t.stats()
            if k >= 2:
                ms.append(st["t_build_ms"] + st["t_total_ms"])
        a = a.cpu().numpy()
        t.free()
        e = np.linalg.norm(a[tg] - bf, axis=1) / np.where(ref > 0, ref, np.median(ref))
        if kw.get("learned"):
            flop = sum(c * 2 * comb(o + 6, 6) for o, c in zip(range(2, 9), st["n_m2l_by_order"]))
        else:
            flop = st["n_m2l"] * 2 * comb(kw["p"] + 6, 6)
        return {"p99": float(np.percentile(e, 99)), "ms": float(np.median(ms)), "pairs": st["p2p_pairs"],
                "m2l_flop": flop}

    forms = {"learned": run(theta=0.5, p=8, learned=1), "plain p8 0.50": run(theta=0.5, p=8),
             "plain p6 0.42": run(theta=0.42, p=6)}
    for k, v in forms.items():
        print("%-14s p99 %.2e  step %.2f ms  P2P pairs %.4e  M2L flop %.4e" % (k, v["p99"], v["ms"], v["pairs"],
                                                                            v["m2l_flop"]))
    best_plain = min(forms["plain p8 0.50"]["ms"], forms["plain p6 0.42"]["ms"])
    print("learned step / best plain step at the same bar: %.3f" % (forms["learned"]["ms"] / best_plain))
    for k, v in forms.items():
        assert v["p99"] <= 1e-3, (k, v)
    assert forms["learned"]["m2l_flop"] < forms["plain p8 0.50"]["m2l_flop"]
    assert forms["learned"]["pairs"] < forms["plain p6 0.42"]["pairs"]
