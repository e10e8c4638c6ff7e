"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Each test names what it pins.  None of them retypes the oracle's own formula: the
references are the paper's printed coefficients, symbolic derivatives (sympy),
high-precision special functions (mpmath), exact algebraic identities, brute force
over all pairs written separately in numpy, and structural invariants."""
import os

import mpmath as mp
import numpy as np
import pytest
import sympy as sp

import oracle
from paper_2006_14952_amd import inputs

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _f_symbolic(kmax, r_val, rs_val):
    """f_(k) = (r^-1 d/dr)^k [erfc(r/2 r_s)/r], by sympy, evaluated with mpmath at 40 digits."""
    r, rs = sp.symbols("r rs", positive=True)
    f = sp.erfc(r / (2 * rs)) / r
    out = []
    for k in range(kmax + 1):
        out.append(float(sp.N(f.subs({r: sp.Rational(r_val), rs: sp.Rational(rs_val)}), 40)))
        f = sp.diff(f, r) / r
    return np.array(out)


# ---- Sec. 2.2 prefactors -----------------------------------------------------

@pytest.mark.parametrize("r,rs", [("1", "1"), ("2", "1"), ("3/10", "1/25"), ("7/5", "3/10"), ("9/2", "1")])
def test_prefactors_match_symbolic_derivatives(r, rs):
    ref = _f_symbolic(8, r, rs)
    rr, rss = float(sp.Rational(r)), float(sp.Rational(rs))
    for method in ("recur", "closed"):
        got = oracle.prefactors(8, rr, rss, method)
        np.testing.assert_allclose(got, ref, rtol=1e-11, err_msg=method)


def test_prefactors_match_paper_printed_coefficients():
    """The explicit f_(2), f_(3), f_(4) printed in Sec. 2.2 (golden file)."""
    rows = [l.split() for l in open(os.path.join(GOLD, "prefactor_coefficients.txt")) if l.strip() and l[0] != "#"]
    for r, rs in [(0.3, 0.11), (1.0, 1.0), (0.05, 0.0390625), (0.17, 0.0390625)]:
        got = oracle.prefactors(4, r, rs, "recur")
        for row in rows:
            k, c, s = int(row[0]), float(row[1]), float(row[2])
            a = [float(v) for v in row[3:]]
            val = c * mp.erfc(r / (2 * rs)) / r ** (2 * k + 1)
            val += s * mp.exp(-r * r / (4 * rs * rs)) / mp.sqrt(mp.pi) * sum(
                a[j] / (rs ** (2 * j + 1) * r ** (2 * k - 2 * j)) for j in range(k))
            assert abs(got[k] - float(val)) <= 1e-12 * abs(float(val)), (k, r, rs)


def test_force_law_closed_form_values():
    """-r^3 f_(1)(r) = erfc(x/2) + x/sqrt(pi) exp(-x^2/4), x = r/r_s (Sec. 2.2 force law),
    evaluated with mpmath."""
    for x in (0.1, 1.0, 2.0, 4.5):
        h = mp.erfc(x / 2) + x / mp.sqrt(mp.pi) * mp.exp(-x * x / 4)
        rs = 0.7
        r = x * rs
        assert abs(-r ** 3 * oracle.f1(r, rs) - float(h)) < 1e-14
        f = oracle.prefactors(1, r, rs)
        assert abs(-r ** 3 * f[1] - float(h)) < 1e-13


def test_newtonian_limit():
    """r_s -> infinity turns every truncated prefactor into Eq. (4)."""
    for r in (0.3, 1.0, 2.5):
        trunc = oracle.prefactors(8, r, 1e7, "recur")
        newt = oracle.prefactors(8, r, 0.0, "newton")
        np.testing.assert_allclose(trunc, newt, rtol=1e-6)
        ref = [(-1) ** k * float(mp.fac2(2 * k - 1)) / r ** (2 * k + 1) for k in range(9)]
        np.testing.assert_allclose(newt, ref, rtol=1e-14)


def test_recurrence_no_cancellation_to_cutoff():
    """Recurrence and closed form agree at every order up to p=10 over (0, 4.5 r_s]."""
    for x in np.linspace(0.05, 4.5, 40):
        a = oracle.prefactors(10, x * 0.01, 0.01, "recur")
        b = oracle.prefactors(10, x * 0.01, 0.01, "closed")
        np.testing.assert_allclose(a, b, rtol=1e-10)


# ---- derivative tensor -----------------------------------------------------------

def test_dtensor_matches_symbolic_gradient():
    X, Y, Z = sp.symbols("X Y Z", real=True)
    rs = sp.Rational(2, 5)
    psi = sp.erfc(sp.sqrt(X ** 2 + Y ** 2 + Z ** 2) / (2 * rs)) / sp.sqrt(X ** 2 + Y ** 2 + Z ** 2)
    R = (sp.Rational(3, 10), sp.Rational(-7, 10), sp.Rational(1, 2))
    p = 5
    D = oracle.dtensor(p, np.array([float(v) for v in R]), float(rs))
    mi = oracle.multi_indices(p)
    for k in [0, 1, 2, 3, 4, 5, 9, 13, 19, 24, 34, 40, 55]:
        n = mi[k]
        e = psi
        for var, cnt in zip((X, Y, Z), n):
            if cnt:
                e = sp.diff(e, var, int(cnt))
        ref = float(sp.N(e.subs({X: R[0], Y: R[1], Z: R[2]}), 30))
        assert abs(D[k] - ref) <= 1e-11 * max(1.0, abs(ref)), (tuple(n), D[k], ref)


def test_dtensor_trace_is_gaussian_source():
    """Poisson: lap[erfc(r/2r_s)/r] = exp(-r^2/4r_s^2)/(2 sqrt(pi) r_s^3) for r > 0, so the
    truncated D_2 is NOT traceless; the Newtonian one is."""
    mi = oracle.multi_indices(2)
    ii = [int(np.where((mi == v).all(axis=1))[0][0]) for v in ([2, 0, 0], [0, 2, 0], [0, 0, 2])]
    for R, rs in [((0.3, -0.7, 0.5), 0.4), ((0.01, 0.02, -0.015), 0.0098)]:
        R = np.array(R)
        r = np.linalg.norm(R)
        D = oracle.dtensor(2, R, rs)
        expect = np.exp(-r * r / (4 * rs * rs)) / (2 * np.sqrt(np.pi) * rs ** 3)
        assert abs(sum(D[i] for i in ii) - expect) < 1e-10 * abs(D[0] / r ** 2)
        Dn = oracle.dtensor(2, R, 0.0)
        assert abs(sum(Dn[i] for i in ii)) < 1e-12 * abs(Dn[0] / r ** 2)


# ---- expansion operators -----------------------------------------------------------

def test_p2m_single_particle_and_m2m_identity():
    rng = np.random.default_rng(11)
    p = 6
    M = oracle.p2m(p, np.array([[0.5, 0.5, 0.5]]), np.array([2.0]), np.array([0.5, 0.5, 0.5]))
    assert M[0] == 2.0 and np.all(M[1:] == 0.0)
    x = rng.random((40, 3)) * 0.01
    mu = rng.random(40)
    zc, zp = np.array([0.004, 0.006, 0.005]), np.array([0.005, 0.005, 0.005])
    a = oracle.m2m(p, oracle.p2m(p, x, mu, zc), zp - zc)
    b = oracle.p2m(p, x, mu, zp)
    np.testing.assert_allclose(a, b, atol=1e-15 * np.abs(b).max())
    # M_{e_x} = -sum mu (x - z)_x  (sign convention of Eq. (1))
    assert abs(b[1] + (mu * (x[:, 0] - zp[0])).sum()) < 1e-15


def test_l2l_is_exact_for_polynomials():
    rng = np.random.default_rng(12)
    p = 7
    L = rng.standard_normal(oracle.ncoef(p))
    shift = np.array([0.3, 0.1, -0.2])
    L2 = oracle.l2l(p, L, shift)
    for _ in range(5):
        y = rng.standard_normal(3) * 0.2
        a = oracle.l2p(p, L, y + shift)
        b = oracle.l2p(p, L2, y)
        assert abs(a[0] - b[0]) < 1e-12
        np.testing.assert_allclose(a[1], b[1], atol=1e-12)


def test_l2p_gradient_matches_potential_differences():
    rng = np.random.default_rng(13)
    p = 5
    L = rng.standard_normal(oracle.ncoef(p))
    y = np.array([0.1, -0.2, 0.05])
    _, g = oracle.l2p(p, L, y)
    h = 1e-6
    for k in range(3):
        e = np.zeros(3); e[k] = h
        num = (oracle.l2p(p, L, y + e)[0] - oracle.l2p(p, L, y - e)[0]) / (2 * h)
        assert abs(num - g[k]) < 1e-7


def _direct_force(x, src, mu, rs):
    g = np.zeros(3)
    for a in range(len(mu)):
        d = x - src[a]
        r = np.linalg.norm(d)
        h = float(mp.erfc(r / (2 * rs)) + r / (rs * mp.sqrt(mp.pi)) * mp.exp(-r * r / (4 * rs * rs)))
        g += -mu[a] * h / r ** 3 * d
    return g


@pytest.mark.parametrize("rs", [0.01, 1e6])
def test_m2l_l2p_converges_to_direct_sum(rs):
    """P2M -> M2L -> L2P approaches the direct truncated sum as p grows (Secs. 2.1-2.2)."""
    rng = np.random.default_rng(1)
    h = 0.01
    src = (rng.random((20, 3)) - 0.5) * h
    mu = rng.random(20)
    zc = np.array([0.025, 0.01, -0.005])
    tgt = zc + (rng.random(3) - 0.5) * h
    ref = _direct_force(tgt, src, mu, rs)
    errs = []
    for p in range(2, 11):
        L = oracle.m2l(p, oracle.p2m(p, src, mu, np.zeros(3)), zc, rs)
        _, g = oracle.l2p(p, L, tgt - zc)
        errs.append(np.linalg.norm(g - ref) / np.linalg.norm(ref))
    assert errs[-1] < 2e-5
    assert all(errs[i + 2] < errs[i] for i in range(len(errs) - 2))


# ---- brute force (the plain definition) --------------------------------------------

def _numpy_all_pairs(pos, mass, rs, rc, G=1.0):
    from scipy.special import erfc
    d = pos[:, None, :] - pos[None, :, :]
    d -= np.round(d)
    r2 = (d ** 2).sum(-1)
    ok = (r2 > 0) & (r2 < rc * rc)
    r = np.sqrt(np.where(ok, r2, 1.0))
    f1 = -(erfc(r / (2 * rs)) + r / (rs * np.sqrt(np.pi)) * np.exp(-r * r / (4 * rs * rs))) / r ** 3
    w = np.where(ok, f1, 0.0) * mass[None, :]
    return G * (w[:, :, None] * d).sum(1)


def test_bruteforce_matches_all_pairs_numpy():
    rng = np.random.default_rng(3)
    pos, m = inputs.clustered(600, 3, rng)
    P = oracle.make_params(rs=0.03, rcut=0.135, G=1.0)
    a = oracle.bruteforce(pos, m, P)
    b = _numpy_all_pairs(pos, m, 0.03, 0.135)
    np.testing.assert_allclose(a, b, rtol=1e-12, atol=1e-12 * np.abs(b).max())
    # momentum: sum m_i a_i = 0 for antisymmetric pair forces
    assert np.abs((m[:, None] * a).sum(0)).max() < 1e-12 * np.abs(m[:, None] * a).sum()


def test_two_body_closed_form():
    rs, rc = 0.04, 0.18
    pos = np.array([[0.5, 0.5, 0.5], [0.5 + 0.06, 0.5 - 0.02, 0.5 + 0.03]])
    m = np.array([0.25, 0.75])
    P = oracle.make_params(rs=rs, rcut=rc, p=4, ncrit=1)
    d = pos[0] - pos[1]
    r = np.linalg.norm(d)
    h = float(mp.erfc(r / (2 * rs)) + r / (rs * mp.sqrt(mp.pi)) * mp.exp(-r * r / (4 * rs * rs)))
    expect0 = -m[1] * h / r ** 3 * d
    for acc in (oracle.bruteforce(pos, m, P), oracle.fmm(pos, m, P).acc):
        np.testing.assert_allclose(acc[0], expect0, rtol=1e-13)
        np.testing.assert_allclose(acc[1], -m[0] / m[1] * expect0, rtol=1e-13)


# ---- the full truncated FMM --------------------------------------------------------

def test_fmm_tiny_theta_equals_bruteforce():
    """With theta -> 0 no pair is ever accepted, every surviving leaf pair is P2P, so the
    traversal's coverage alone decides the result: it must equal brute force."""
    rng = np.random.default_rng(4)
    pos, m = inputs.clustered(3000, 4, rng)
    P = oracle.make_params(rs=0.02, rcut=0.09, theta=1e-3, p=2, ncrit=8)
    res = oracle.fmm(pos, m, P)
    assert res.stats["n_m2l"] == 0
    bf = oracle.bruteforce(pos, m, P)
    np.testing.assert_allclose(res.acc, bf, rtol=1e-10, atol=1e-12 * np.abs(bf).max())


def test_fmm_uniform_strict_mac_has_no_m2l_and_is_exact():
    """Uniform 32^3 with r_s = 1.25 cells: every surviving pair straddles the cutoff, so
    the strict transition rule leaves only P2P (M2L vanishes in the uniform case, Sec. 3)."""
    pos, m = inputs.make("uniform")
    pr = inputs.split_params("uniform")
    P = oracle.make_params(rs=pr["rs"], rcut=pr["rcut"], theta=0.5, p=4, ncrit=32)
    res = oracle.fmm(pos, m, P)
    assert res.stats["n_m2l"] == 0
    tg = np.arange(0, len(pos), 7)
    bf = oracle.bruteforce(pos, m, P, targets=tg)
    np.testing.assert_allclose(res.acc[tg], bf, rtol=1e-10, atol=1e-13 * np.abs(bf).max())


def _rel_err(a, b):
    """|a - b| / |b|; particles with no neighbour inside r_cut (|b| = 0) are scored by
    |a| against the typical force scale instead (they must come out as zero)."""
    nb = np.linalg.norm(b, axis=1)
    floor = np.median(nb[nb > 0])
    return np.linalg.norm(a - b, axis=1) / np.where(nb > 0, nb, floor)


def test_fmm_error_falls_with_order_and_theta():
    rng = np.random.default_rng(6)
    pos, m = inputs.clustered(20000, 12, rng)
    bf = oracle.bruteforce(pos, m, oracle.make_params(rs=0.01, rcut=0.045))
    e = {}
    for p, th in [(2, 0.5), (4, 0.5), (6, 0.5), (8, 0.5), (6, 0.3)]:
        P = oracle.make_params(rs=0.01, rcut=0.045, theta=th, p=p, ncrit=16)
        res = oracle.fmm(pos, m, P)
        assert res.stats["n_m2l"] > 0
        e[(p, th)] = np.percentile(_rel_err(res.acc, bf), 99)
    assert e[(2, 0.5)] > e[(4, 0.5)] > e[(6, 0.5)] > e[(8, 0.5)]
    assert e[(6, 0.3)] < e[(6, 0.5)]
    assert e[(8, 0.5)] < 1e-3


def test_literal_rules_are_worse():
    """mac_mode 1 (literal S_c test of item 3) and mac_mode 2 (source-only size in item 2)
    give larger errors than the default strict reading at the same p, theta."""
    rng = np.random.default_rng(7)
    pos, m = inputs.clustered(20000, 12, rng)
    bf = oracle.bruteforce(pos, m, oracle.make_params(rs=0.01, rcut=0.045))
    e = []
    for mode in (0, 1, 2):
        P = oracle.make_params(rs=0.01, rcut=0.045, theta=0.5, p=6, ncrit=16, mac_mode=mode)
        e.append(np.percentile(_rel_err(oracle.fmm(pos, m, P).acc, bf), 99))
    assert e[0] < e[1] and e[0] < e[2]


def test_fmm_lattice_zero_force_and_momentum():
    pos, m = inputs.lattice(16)
    P = oracle.make_params(rs=1.25 / 16, rcut=4.5 * 1.25 / 16, theta=0.5, p=4, ncrit=8)
    res = oracle.fmm(pos, m, P)
    scale = m[0] / (1.0 / 16) ** 2
    assert np.abs(res.acc).max() < 1e-10 * scale
    rng = np.random.default_rng(8)
    pos, m = inputs.clustered(8000, 6, rng)
    P = oracle.make_params(rs=0.015, rcut=0.0675, theta=0.4, p=6, ncrit=16)
    acc = oracle.fmm(pos, m, P).acc
    tot = np.abs(m[:, None] * acc).sum()
    assert np.abs((m[:, None] * acc).sum(0)).max() < 1e-4 * tot


def _cells_table(res):
    cells = res.cells()
    return {int(k): (int(b), int(e)) for k, lvl, b, e, nc in cells}


def test_interaction_lists_partition_pairs():
    """Every particle pair (i, j) within r_cut is covered exactly once: by a P2P leaf pair
    or by an M2L cell pair whose cells contain i and j, with the image of the pair."""
    rng = np.random.default_rng(9)
    pos, m = inputs.clustered(1500, 3, rng)
    P = oracle.make_params(rs=0.03, rcut=0.135, theta=0.5, p=3, ncrit=4)
    res = oracle.fmm(pos, m, P)
    cells = res.cells()
    orig = np.zeros(len(pos), np.int64)
    oracle.lib().orc_copy_cells(res._h, cells, orig.ctypes.data)
    where = np.empty_like(orig)
    where[orig] = np.arange(len(orig))
    rng_of = {int(k): (int(b), int(e)) for k, _, b, e, _ in cells}
    cover = {}
    for kind in ("p2p", "m2l"):
        for a, b, s in res.lists(kind):
            ba, ea = rng_of[int(a)]
            bb, eb = rng_of[int(b)]
            for i in range(ba, ea):
                for j in range(bb, eb):
                    key = (i, j, int(s))
                    cover[key] = cover.get(key, 0) + 1
    assert max(cover.values()) == 1
    x = np.mod(pos, 1.0)[orig]
    n = len(x)
    need = 0
    for i in range(n):
        d = x[i] - x
        img = np.round(d).astype(int)
        r2 = ((d - img) ** 2).sum(1)
        for j in np.nonzero(r2 < P.rcut ** 2)[0]:
            if j == i:
                continue
            s = (img[j, 0] + 1) * 9 + (img[j, 1] + 1) * 3 + (img[j, 2] + 1)
            assert cover.get((i, int(j), int(s)), 0) == 1, (i, j, s)
            need += 1
    assert need > 1000


# ---- conventional MAC (mac_mode bit 2), the baseline of the cost comparison of Sec. 3 --

def test_conventional_mac_tiny_theta_lists_every_leaf_pair():
    """Conventional MAC, theta -> 0: nothing is accepted or neglected, so every pair of
    leaves in every one of the 27 root images becomes a P2P pair (27 nleaf^2 of them) and
    the forces are the hard-cut sum."""
    rng = np.random.default_rng(41)
    pos, m = inputs.clustered(300, 2, rng)
    P = oracle.make_params(rs=0.03, rcut=0.135, theta=1e-3, p=2, ncrit=8, mac_mode=4)
    res = oracle.fmm(pos, m, P)
    nleaf = res.stats["nleaf"]
    assert res.stats["n_m2l"] == 0
    assert res.stats["n_p2p"] == 27 * nleaf * nleaf
    bf = oracle.bruteforce(pos, m, P)
    np.testing.assert_allclose(res.acc, bf, rtol=1e-10, atol=1e-12 * np.abs(bf).max())


def test_conventional_mac_covers_every_pair_of_every_image_once():
    """Without the neglect rule the lists cover all particle pairs of all 27 images (not
    only those inside r_cut), each exactly once, by P2P or by M2L."""
    rng = np.random.default_rng(42)
    pos, m = inputs.clustered(150, 2, rng)
    P = oracle.make_params(rs=0.03, rcut=0.135, theta=0.5, p=3, ncrit=4, mac_mode=4)
    res = oracle.fmm(pos, m, P)
    assert res.stats["n_m2l"] > 0
    rng_of = {int(k): (int(b), int(e)) for k, _, b, e, _ in res.cells()}
    seen = np.zeros((len(pos), len(pos), 27), np.int64)
    for kind in ("p2p", "m2l"):
        for a, b, s in res.lists(kind):
            ba, ea = rng_of[int(a)]
            bb, eb = rng_of[int(b)]
            seen[ba:ea, bb:eb, int(s)] += 1
    assert seen.min() == 1 and seen.max() == 1


def test_uniform_m2l_vanishes_only_with_the_truncated_mac():
    """Uniform 32^3 box, r_s = 1.25 mesh cells, leaves of up to 32 particles (Sec. 3): the
    truncated MAC leaves no M2L at all (every surviving pair is handled by P2P, as in P3M),
    the conventional MAC needs many.  Here every leaf lies on one level, so the
    conventional MAC opens exactly the 27 adjacent leaves of each leaf (L / S_c = 1) and
    accepts every pair two cells apart (L / S_c = 1/2 = theta).  The leaves are the
    occupied cells of the 16^3 grid (counted here from the positions): the conventional
    P2P count is the number of ordered pairs of occupied cells that are periodic
    neighbours (each cell with itself included)."""
    pos, m = inputs.make("uniform")
    pr = inputs.split_params("uniform")
    kw = dict(rs=pr["rs"], rcut=pr["rcut"], theta=0.5, p=2, ncrit=32)
    tr = oracle.fmm(pos, m, oracle.make_params(**kw)).stats
    cv = oracle.fmm(pos, m, oracle.make_params(mac_mode=4, **kw)).stats
    assert tr["n_m2l"] == 0 and tr["n_p2p"] > 0
    assert cv["n_m2l"] > 1000
    c3 = np.bincount(np.ravel_multi_index(np.floor(pos * 8).astype(int).T, (8, 8, 8)), minlength=512)
    assert c3.min() > 32  # every level-3 cell splits, no level-4 cell does (count <= 32 below)
    c4 = np.bincount(np.ravel_multi_index(np.floor(pos * 16).astype(int).T, (16, 16, 16)),
                     minlength=4096).reshape(16, 16, 16)
    assert c4.max() <= 32
    occ = c4 > 0
    assert cv["nleaf"] == occ.sum() and cv["maxlevel"] == 4
    neigh = sum(np.roll(occ, (dx, dy, dz), axis=(0, 1, 2)).astype(int)
                for dx in (-1, 0, 1) for dy in (-1, 0, 1) for dz in (-1, 0, 1))
    assert cv["n_p2p"] == int((neigh * occ).sum())


# ---- polynomial split (the alternative truncation function of Sec. 5) ------------------

def _poly_g_symbolic():
    """g(x) = 1 - x h(x^2) of lowest degree with g(1) = g'(1) = g''(1) = 0, solved by sympy
    from those conditions (so the coefficients are not retyped)."""
    x, a0, a1, a2 = sp.symbols("x a0 a1 a2")
    g = 1 - x * (a0 + a1 * x ** 2 + a2 * x ** 4)
    sol = sp.solve([g.subs(x, 1), sp.diff(g, x).subs(x, 1), sp.diff(g, x, 2).subs(x, 1)], [a0, a1, a2])
    return x, g.subs(sol)


def test_poly_split_prefactors_match_symbolic_derivatives():
    x, g = _poly_g_symbolic()
    r, rc = sp.symbols("r rc", positive=True)
    f = g.subs(x, r / rc) / r
    for rv, rcv in [("1/10", "1"), ("1/2", "1"), ("9/10", "1"), ("3/100", "1/20"), ("7/5", "2")]:
        got = oracle.prefactors(8, float(sp.Rational(rv)), 0.0, "poly", rc=float(sp.Rational(rcv)))
        e = f
        for k in range(9):
            ref = float(sp.N(e.subs({r: sp.Rational(rv), rc: sp.Rational(rcv)}), 40))
            assert abs(got[k] - ref) <= 1e-11 * max(abs(ref), 1e-300), (k, rv, got[k], ref)
            e = sp.diff(e, r) / r


def test_poly_split_vanishes_smoothly_and_long_range_is_regular():
    """phi_s and its force vanish at r_cut; the long range (1 - g)/r is even in r (finite,
    with zero slope, at r = 0)."""
    x, g = _poly_g_symbolic()
    assert sp.simplify(g.subs(x, 1)) == 0 and sp.simplify(sp.diff(g, x).subs(x, 1)) == 0
    lr = sp.expand((1 - g) / x)
    assert all(int(t.as_poly(x).degree()) % 2 == 0 for t in lr.as_ordered_terms())
    rc = 0.3
    for r in (rc * (1 - 1e-7),):
        f = oracle.prefactors(1, r, 0.0, "poly", rc=rc)
        assert abs(f[0]) * r < 1e-12 and abs(oracle.f1_poly(r, rc)) * r ** 3 < 1e-12
    np.testing.assert_allclose(oracle.f1_poly(0.1, rc), oracle.prefactors(1, 0.1, 0.0, "poly", rc=rc)[1], rtol=1e-14)


def test_poly_split_dtensor_matches_symbolic_gradient():
    xs, g = _poly_g_symbolic()
    X, Y, Z = sp.symbols("X Y Z", real=True)
    rc = sp.Rational(3, 2)
    rr = sp.sqrt(X ** 2 + Y ** 2 + Z ** 2)
    psi = g.subs(xs, rr / rc) / rr
    R = (sp.Rational(3, 10), sp.Rational(-7, 10), sp.Rational(1, 2))
    p = 5
    D = oracle.dtensor(p, np.array([float(v) for v in R]), 0.0, split=1, rc=float(rc))
    mi = oracle.multi_indices(p)
    for k in [0, 1, 2, 3, 4, 5, 9, 13, 19, 24, 34, 40, 55]:
        n = mi[k]
        e = psi
        for var, cnt in zip((X, Y, Z), n):
            if cnt:
                e = sp.diff(e, var, int(cnt))
        ref = float(sp.N(e.subs({X: R[0], Y: R[1], Z: R[2]}), 30))
        assert abs(D[k] - ref) <= 1e-11 * max(1.0, abs(ref)), (tuple(n), D[k], ref)


def test_poly_split_fmm_tiny_theta_equals_bruteforce_and_error_falls_with_order():
    rng = np.random.default_rng(44)
    pos, m = inputs.clustered(3000, 4, rng)
    P = oracle.make_params(rs=0.0, rcut=0.09, theta=1e-3, p=2, ncrit=8, split=1)
    res = oracle.fmm(pos, m, P)
    assert res.stats["n_m2l"] == 0
    bf = oracle.bruteforce(pos, m, P)
    np.testing.assert_allclose(res.acc, bf, rtol=1e-10, atol=1e-12 * np.abs(bf).max())
    pos, m = inputs.clustered(20000, 12, np.random.default_rng(45))
    bf = oracle.bruteforce(pos, m, oracle.make_params(rs=0.0, rcut=0.045, split=1))
    e = []
    for p in (2, 4, 6):
        res = oracle.fmm(pos, m, oracle.make_params(rs=0.0, rcut=0.045, theta=0.5, p=p, ncrit=16, split=1))
        assert res.stats["n_m2l"] > 0
        e.append(np.percentile(_rel_err(res.acc, bf), 99))
    assert e[0] > e[1] > e[2]
