"""The paper's two measurements (error against opening angle; truncated against
conventional interaction counts) as computed by the library, checked against the
oracle's counts and brute force on small inputs."""
import numpy as np
import pytest

import oracle
from paper_2006_14952_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
ex = pytest.importorskip("paper_2006_14952_amd.experiments")


def test_interaction_counts_match_oracle_and_levels_add_up():
    pos, m = inputs.lattice(16)
    rng = inputs.rng_for(120)
    pos = np.mod(pos + rng.uniform(-0.5, 0.5, pos.shape) / 16, 1.0)
    rs, rc = 1.25 / 16, 4.5 * 1.25 / 16
    # every MAC form the experiment reports: the library default, the paper's source-side
    # size with the strict and the literal item 3, and the two conventional forms
    modes = tuple(ex.MAC_MODES)
    assert set(modes) == {0, 2, 3, 4, 6}
    rows = ex.interaction_counts(pos, m, rs, rc, theta=0.5, p=3, n_crits=(1, 8), modes=modes)
    assert len(rows) == 2 * len(modes)
    for r in rows:
        ref = oracle.fmm(pos, m, oracle.make_params(rs=rs, rcut=rc, theta=0.5, p=3, ncrit=r["n_crit"],
                                                    mac_mode=r["mac_mode"])).stats
        assert r["n_m2l"] == ref["n_m2l"] and r["n_p2p"] == ref["n_p2p"], r
        assert r["p2p_pairs"] == ref["p2p_pairs"], r
        assert sum(r["m2l_per_level"]) == r["n_m2l"] and sum(r["p2p_per_level"]) == r["n_p2p"]


def test_error_vs_theta_reference_is_the_hard_cut_sum_and_error_grows_with_theta():
    rng = inputs.rng_for(121)
    pos, m = inputs.clustered(20000, 12, rng)
    rs, rc = 0.01, 0.045
    for mode in (0, 2, 3):
        rows = ex.error_vs_theta(pos, m, rs, rc, [0.2, 0.5, 0.8], p=4, n_crit=16, mac_mode=mode)
        assert rows[0]["rms"] < rows[1]["rms"] < rows[2]["rms"], (mode, rows)
        if mode == 0:  # with the source side alone, small sources pass item 2 at any theta
            assert rows[0]["n_m2l"] < rows[2]["n_m2l"]
    # the theta -> 0 reference equals brute force
    ref, st, t = ex._forces(pos, m, ex.params(r_s=rs, r_cut=rc, theta=1e-3, p=4, n_crit=16))
    t.free()
    assert st["n_m2l"] == 0
    bf = oracle.bruteforce(pos, m, oracle.make_params(rs=rs, rcut=rc))
    np.testing.assert_allclose(ref, bf, rtol=1e-9, atol=1e-12 * np.abs(bf).max())
