"""Pins of the long-range CPU references (PM and Ewald)."""
import numpy as np
import pytest

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


def test_poly_split_window_is_the_transform_of_its_density():
    """The polynomial split's long-range Fourier factor against a quadrature of its
    smoothing density 15/(8 pi r_c^3)(1 - r^2/r_c^2) over r < r_c."""
    from scipy.integrate import quad
    rc = 0.2
    for k in (0.0, 0.3, 4.0, 25.0, 90.0, 300.0):
        num = quad(lambda r: 15 / (8 * np.pi * rc ** 3) * (1 - r * r / rc ** 2) * 4 * np.pi * r * r *
                   (np.sinc(k * r / np.pi) if k > 0 else 1.0), 0.0, rc, limit=200)[0]
        got = pm_ewald.long_range_window(np.array([k]), split=1, rcut=rc)[0]
        assert abs(got - num) < 1e-10, (k, got, num)


def test_poly_split_pm_plus_short_range_is_newtonian():
    """PM with the polynomial split's window plus its short-range pair sum gives the
    periodic Newtonian force (Ewald).  The polynomial split has compact support, so it
    loses nothing at r_cut, while the Gaussian split's hard cut drops the erfc tail
    (rms 2.5e-5 against 2.0e-4 here)."""
    from oracle import bruteforce, make_params
    rng = inputs.rng_for(204)
    pos, m = inputs.clustered(3000, 4, rng)
    M = 64
    rs = 1.25 / M
    rc = 4.5 * rs
    ew = pm_ewald.ewald_total(pos, m, 1.0, rs)
    scale = np.sqrt((ew ** 2).sum(1).mean())
    tot = {}
    for split in (0, 1):
        pm = pm_ewald.pm_forces(pos, m, 1.0, rs, M, split=split, rcut=rc)
        sr = bruteforce(pos, m, make_params(rs=rs, rcut=rc, split=split))
        tot[split] = np.sqrt(((pm + sr - ew) ** 2).sum(1).mean()) / scale
    assert tot[1] < 1e-4 and tot[0] < 1e-3 and tot[1] < tot[0], tot


@pytest.mark.parametrize("order", [2, 3, 4])
def test_assignment_weights_are_the_b_spline_of_their_order(order):
    """Each weight equals the order-p B-spline (p-fold convolution of the unit box,
    formed here numerically on a fine grid) at the node's distance from the particle;
    the weights sum to 1 and keep the particle's position as their mean."""
    from scipy.signal import fftconvolve
    h = 1e-4
    box1 = np.ones(int(round(1 / h)))
    spline = box1.copy()
    for _ in range(order - 1):
        spline = fftconvolve(spline, box1) * h
    xs = (np.arange(len(spline)) + 0.5) * h - order / 2.0  # support [-p/2, p/2]
    rng = inputs.rng_for(205, order)
    M = 16
    pos = rng.random((500, 3))
    first, w = pm_ewald.assignment(pos, 1.0, M, order)
    g = pos * M - 0.5                                      # particle in node units
    np.testing.assert_allclose(w.sum(-1), 1.0, atol=1e-14)
    nodes = first[:, :, None] + np.arange(order)          # mod M: unwrap by the nearest image
    d = (nodes - g[:, :, None] + M / 2) % M - M / 2
    np.testing.assert_allclose((w * (g[:, :, None] + d)).sum(-1), g, atol=1e-12)
    np.testing.assert_allclose(w, np.interp(d, xs, spline), atol=5e-4)
    assert np.all(np.abs(d) <= order / 2.0 + 1e-12)


def test_higher_order_assignment_brings_pm_closer_to_ewald():
    """The PM step approximates the reciprocal Ewald sum; with the window divided out,
    its aliasing error falls as the assignment order rises (CIC > TSC > PCS)."""
    rng = inputs.rng_for(206)
    pos, m = inputs.clustered(3000, 4, rng)
    M = 32
    rs = 1.25 / M
    ew = pm_ewald.ewald_reciprocal(pos, m, 1.0, rs)
    err = {}
    for order in (2, 3, 4):
        pm = pm_ewald.pm_forces(pos, m, 1.0, rs, M, order=order)
        err[order] = np.sqrt(((pm - ew) ** 2).sum(1).mean() / (ew ** 2).sum(1).mean())
    assert err[2] > err[3] > err[4], err
    assert err[4] < 0.5 * err[2], err
