"""GPU parity at the two largest workloads, at full size and in the launch configurations
bench.py times (each leaf limit its autotuner chooses from), on sampled particles the CPU
side can afford:

* 256^3 clustered (8000 clumps), order 8, theta 0.5, FP32: plain form against the FP64
  oracle on sampled particles (only their sink cells are traversed on the CPU) and against
  the brute-force sum; the learned selector against the brute-force sum.
* 512^3 lattice + 32000 clumps, full hybrid step with the learned selector: short-range
  part against the brute-force sum on sampled particles, and the total equal to the PM
  part plus the short-range part (the PM step itself is checked against its CPU reference
  at smaller meshes in test_gpu_pm_batched.py)."""
import os

import numpy as np
import pytest

import oracle
from helpers import rel_err
from paper_2006_14952_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
hf = pytest.importorskip("paper_2006_14952_amd")
from paper_2006_14952_amd import learned  # noqa: E402


def _bf_err(got, pos, m, op, tg):
    bf = oracle.bruteforce(pos, m, op, targets=tg)
    ref = np.linalg.norm(bf, axis=1)
    return np.linalg.norm(got[tg] - bf, axis=1) / np.where(ref > 0, ref, np.median(ref))


def _leaf_limits(workload):
    import bench
    return bench.WORKLOADS[workload]["tune"]


@pytest.mark.parametrize("ncrit", _leaf_limits("large"))
def test_large_config_full_size_sampled(ncrit):
    print("case: 16.7M box, n_crit %d" % ncrit, flush=True)
    pos, m = inputs.make("large")
    pr = inputs.split_params("large")
    n = len(pos)
    tg = inputs.rng_for(3, 11).choice(n, 600, replace=False)
    dp, dm = torch.tensor(pos, device="cuda"), torch.tensor(m, device="cuda")
    prm = hf.params(r_s=pr["rs"], r_cut=pr["rcut"], theta=0.5, p=8, n_crit=ncrit, precision=1)
    t = hf.Tree().build(dp, dm, prm)
    got = t.short_range(prm).cpu().numpy()
    st = t.stats()
    t.free()
    op = oracle.make_params(box=1.0, rs=pr["rs"], rcut=pr["rcut"], theta=0.5, p=8, ncrit=ncrit)
    ref = oracle.fmm(pos, m, op, targets=tg)
    e_or = rel_err(got[tg], ref.acc[tg])
    print("large plain, n_crit %d: median %.2e p99 %.2e max %.2e vs oracle" % (
        ncrit, np.median(e_or), np.percentile(e_or, 99), e_or.max()))
    assert np.median(e_or) <= 1e-6 and np.percentile(e_or, 99) <= 1e-4
    assert st["p2p_evaluated"] <= st["p2p_pairs"]
    assert np.percentile(_bf_err(got, pos, m, op, tg), 99) <= 1e-3
    if os.path.exists(learned.DEFAULT_MODEL):
        learned.load_model()
        prm.learned = 1
        t = hf.Tree().build(dp, dm, prm)
        got_l = t.short_range(prm).cpu().numpy()
        st_l = t.stats()
        t.free()
        assert sum(st_l["n_m2l_by_order"]) == st_l["n_m2l"] > 0
        e_l = _bf_err(got_l, pos, m, op, tg)
        print("large learned: p99 %.2e vs brute force" % np.percentile(e_l, 99))
        assert np.percentile(e_l, 99) <= 1e-3


@pytest.mark.parametrize("ncrit", _leaf_limits("full"))
def test_full_config_hybrid_sampled(ncrit):
    print("case: 134M box hybrid, n_crit %d" % ncrit, flush=True)
    if not os.path.exists(learned.DEFAULT_MODEL):
        pytest.skip("no trained model file")
    pos, m = inputs.make("full")
    pr = inputs.split_params("full")
    mesh = inputs.CONFIGS["full"]["mesh"]
    n = len(pos)
    tg = inputs.rng_for(4, 11).choice(n, 1500, replace=False)
    dp, dm = torch.tensor(pos, device="cuda"), torch.tensor(m, device="cuda")
    learned.load_model()
    prm = hf.params(r_s=pr["rs"], r_cut=pr["rcut"], theta=0.5, p=8, n_crit=ncrit, precision=1, learned=1)
    t = hf.Tree()
    tot = t.hybrid(dp, dm, prm, mesh)
    sr = t.short_range(prm)
    t.free()
    lr = hf.pm_long_range(dp, dm, prm, mesh)
    # the two short-range evaluations differ by FP32 rounding (atomic order in M2L)
    d = (tot - sr - lr).norm(dim=1)
    assert (d / tot.norm(dim=1).clamp_min(1e-300)).median().item() <= 1e-6
    op = oracle.make_params(box=1.0, rs=pr["rs"], rcut=pr["rcut"], theta=0.5, p=8, ncrit=ncrit)
    e = _bf_err(sr.cpu().numpy(), pos, m, op, tg)
    print("full hybrid, n_crit %d: short range p99 %.2e vs brute force" % (ncrit, np.percentile(e, 99)))
    assert np.percentile(e, 99) <= 1e-3
