"""Pins of the long-range CPU references (PM and Ewald)."""
import numpy as np

from oracle import pm_ewald
from paper_2006_14952_amd import inputs


def test_ewald_total_is_independent_of_split_scale():
    """Real + reciprocal Ewald sums give the periodic Newtonian force whatever alpha is:
    a wrong factor, sign or term in either part breaks the agreement."""
    rng = inputs.rng_for(201)
    pos = rng.random((40, 3))
    m = rng.random(40) / 40
    a = pm_ewald.ewald_total(pos, m, 1.0, 0.02)
    b = pm_ewald.ewald_total(pos, m, 1.0, 0.035)
    np.testing.assert_allclose(a, b, rtol=1e-8, atol=1e-10 * np.abs(a).max())


def test_ewald_lattice_zero_and_momentum():
    pos, m = inputs.lattice(4)
    a = pm_ewald.ewald_total(pos, m, 1.0, 0.03)
    assert np.abs(a).max() < 1e-10
    rng = inputs.rng_for(202)
    pos = rng.random((60, 3))
    m = np.full(60, 1 / 60)
    a = pm_ewald.ewald_total(pos, m, 1.0, 0.03)
    assert np.abs((m[:, None] * a).sum(0)).max() < 1e-10 * np.abs(m[:, None] * a).sum()


def test_ewald_two_close_particles_match_newton():
    """At a separation much smaller than the box the periodic force tends to the
    Newtonian pair force (images contribute O(d/L^3))."""
    pos = np.array([[0.5, 0.5, 0.5], [0.5 + 1e-3, 0.5, 0.5]])
    m = np.array([1.0, 1.0])
    a = pm_ewald.ewald_total(pos, m, 1.0, 0.02)
    newton = 1.0 / 1e-6
    assert abs(a[0, 0] - newton) / newton < 1e-4
    assert abs(a[1, 0] + newton) / newton < 1e-4


def test_pm_reference_matches_ewald_reciprocal():
    rng = inputs.rng_for(203)
    pos, m = inputs.clustered(3000, 4, rng)
    M = 64
    rs = 1.25 / M
    pm = pm_ewald.pm_forces(pos, m, 1.0, rs, M)
    ew = pm_ewald.ewald_reciprocal(pos, m, 1.0, rs)
    rms = np.sqrt(((pm - ew) ** 2).sum(1).mean() / (ew ** 2).sum(1).mean())
    assert rms < 2e-2, rms
