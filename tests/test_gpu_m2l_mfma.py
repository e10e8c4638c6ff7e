"""The matrix-core M2L (pairs of cells on one level as FP32 MFMA products, fmm_params
m2l_mfma = 2) against the FP64 oracle and against the lane-per-pair VALU kernel
(m2l_mfma = 1), at every order it covers, with long lists (windows sorted in several
chunks), deep trees (pairs below level 15 stay on the VALU kernel) and a full-size box."""
import numpy as np
import pytest

import oracle
from helpers import rel_err
from paper_2006_14952_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
hf = pytest.importorskip("paper_2006_14952_amd")


def run(pos, m, prm, tree=None):
    t = tree or hf.Tree()
    t.build(torch.tensor(pos, device="cuda"), torch.tensor(m, device="cuda"), prm)
    acc = t.short_range(prm).cpu().numpy()
    st = t.stats()
    if tree is None:
        t.free()
    return acc, st


def opar(prm):
    return oracle.make_params(box=prm.box, rs=prm.r_s, rcut=prm.r_cut, theta=prm.theta, p=prm.p, ncrit=prm.n_crit)


@pytest.mark.parametrize("p", [4, 5, 6, 7, 8])
def test_mfma_m2l_matches_oracle_and_valu_kernel(p):
    pos, m = inputs.clustered(60000, 60, inputs.rng_for(150, p))
    prm = hf.params(r_s=0.01, r_cut=0.045, theta=0.4, p=p, n_crit=32, precision=1, m2l_mfma=2)
    got, st = run(pos, m, prm)
    prm.m2l_mfma = 1
    valu, st1 = run(pos, m, prm)
    assert st["n_m2l"] == st1["n_m2l"] and st["n_m2l"] > 10000
    ref = oracle.fmm(pos, m, opar(prm)).acc
    e = rel_err(got, ref)
    e1 = rel_err(valu, ref)
    print("p=%d mfma vs oracle: median %.2e p99 %.2e max %.2e (valu: %.2e %.2e %.2e)" % (
        p, np.median(e), np.percentile(e, 99), e.max(), np.median(e1), np.percentile(e1, 99), e1.max()))
    assert np.median(e) <= 1e-6 and np.percentile(e, 99) <= 2e-5 and e.max() <= 1e-3
    # the two kernels add the same terms in another order: FP32 rounding apart
    assert np.percentile(rel_err(got, valu), 99) <= 2e-5


def test_mfma_m2l_long_lists_and_deep_levels():
    """A small opening angle gives every sink long M2L lists (a window's pairs are sorted
    in several chunks of 2048); a very compact clump puts cells below level 15 (their
    pairs stay on the VALU kernel)."""
    rng = inputs.rng_for(151)
    pos, m = inputs.clustered(40000, 20, rng)
    blob = 0.5 + rng.normal(scale=2e-6, size=(4000, 3))  # cells to about level 19
    pos = np.concatenate([pos, blob])
    m = np.full(len(pos), 1.0 / len(pos))
    prm = hf.params(r_s=0.008, r_cut=0.036, theta=0.25, p=6, n_crit=4, precision=1, m2l_mfma=2)
    got, st = run(pos, m, prm)
    assert st["max_level"] > 15
    prm.m2l_mfma = 1
    valu, _ = run(pos, m, prm)
    ref = oracle.fmm(pos, m, opar(prm)).acc
    e = rel_err(got, ref)
    print("long lists: M2L pairs %d (%.0f per sink cell)  mfma vs oracle median %.2e p99 %.2e max %.2e" % (
        st["n_m2l"], st["n_m2l"] / st["n_cells"], np.median(e), np.percentile(e, 99), e.max()))
    assert st["n_m2l"] / st["n_cells"] > 40
    assert np.median(e) <= 1e-6 and np.percentile(e, 99) <= 2e-5
    assert np.percentile(rel_err(got, valu), 99) <= 2e-5


def test_mfma_m2l_full_size_order_8_sampled():
    """N = 256^3 clustered at order 8 with the plain MAC (the order-8 M2L is the largest
    stage there): FP32 with the matrix-core M2L against the FP64 oracle on sampled
    particles, and against the VALU kernel everywhere."""
    pos, m = inputs.make("large")
    pr = inputs.split_params("large")
    tg = inputs.rng_for(4, 12).choice(len(pos), 600, replace=False)
    prm = hf.params(r_s=pr["rs"], r_cut=pr["rcut"], theta=0.5, p=8, n_crit=32, precision=1, m2l_mfma=2)
    t = hf.Tree()
    got, st = run(pos, m, prm, t)
    prm.m2l_mfma = 1
    valu, _ = run(pos, m, prm, t)
    t.free()
    ref = oracle.fmm(pos, m, opar(prm), targets=tg).acc
    e = rel_err(got[tg], ref[tg])
    print("16.7M order 8: mfma vs oracle median %.2e p99 %.2e max %.2e" % (np.median(e), np.percentile(e, 99), e.max()))
    assert np.median(e) <= 1e-6 and np.percentile(e, 99) <= 2e-5
    assert np.percentile(rel_err(got, valu), 99) <= 2e-5
