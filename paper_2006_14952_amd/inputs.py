"""Seeded synthetic particle sets and the five workload configurations.

This module holds no arithmetic of the method: it only draws positions and masses.
It is the one module that both the GPU library's callers and the CPU oracle's tests
use, so that both sides see bit-identical inputs.

Workloads (periodic unit box, G = 1, equal masses 1/N per box):
  uniform    N = 32^3 uniform random                                   (plain FP64 form)
  clustered  N = 128^3: 50% uniform background, 50% in 2000 Hernquist
             spheres (scale radii log-uniform 0.002-0.02, clump masses
             dN/dM ~ M^-1.9 on [1, 1e3])                               (FP32 form)
  batched    64 boxes, N_b = round(2^U(12,18)), each a clustered mix   (batched FP32 form)
  large      N = 256^3 clustered with 8000 clumps                      (learned-MAC form)
  full       N = 512^3 displaced lattice, a 50% subset moved into
             32000 clumps                                              (full-size form)
The paper's clustered input (a LCDM z=0 snapshot) is not available; the Hernquist
mixtures stand in for its shape.  Splitting scale r_s = 1.25 mesh cells and cutoff
r_cut = 4.5 r_s follow the paper's r_s ~ 1.2 grid cells and ~5 r_s truncation.
"""
from __future__ import annotations

import numpy as np

SEED = 2006_14952


def rng_for(*key):
    return np.random.default_rng([SEED, *key])


def uniform(n, rng, box=1.0):
    pos = rng.random((n, 3)) * box
    return pos, np.full(n, 1.0 / n)


def _largest_remainder(weights, total):
    w = np.asarray(weights, np.float64)
    share = w / w.sum() * total
    base = np.floor(share).astype(np.int64)
    left = int(total - base.sum())
    if left > 0:
        order = np.argsort(-(share - base), kind="stable")
        base[order[:left]] += 1
    return base


def hernquist_clumps(n, n_clumps, rng, box=1.0, a_min=0.002, a_max=0.02, m_lo=1.0, m_hi=1e3, slope=-1.9,
                     rmax_over_a=10.0):
    """n particles in n_clumps truncated Hernquist spheres with uniform centres."""
    centres = rng.random((n_clumps, 3)) * box
    a = np.exp(rng.uniform(np.log(a_min), np.log(a_max), n_clumps))
    g = slope + 1.0                                   # inverse CDF of dN/dM ~ M^slope
    u = rng.random(n_clumps)
    mclump = (m_lo ** g + u * (m_hi ** g - m_lo ** g)) ** (1.0 / g)
    counts = _largest_remainder(mclump, n)
    cid = np.repeat(np.arange(n_clumps), counts)
    ai = a[cid]
    umax = (rmax_over_a / (rmax_over_a + 1.0)) ** 2   # M(<r) ~ r^2/(r+a)^2, truncated at rmax
    q = np.sqrt(rng.random(n) * umax)
    r = ai * q / (1.0 - q)
    cth = rng.uniform(-1.0, 1.0, n)
    phi = rng.uniform(0.0, 2.0 * np.pi, n)
    sth = np.sqrt(np.maximum(0.0, 1.0 - cth * cth))
    d = np.stack([sth * np.cos(phi), sth * np.sin(phi), cth], axis=1)
    pos = centres[cid] + r[:, None] * d
    return np.mod(pos, box)


def clustered(n, n_clumps, rng, box=1.0, frac=0.5):
    n_cl = int(round(frac * n))
    bg = rng.random((n - n_cl, 3)) * box
    cl = hernquist_clumps(n_cl, n_clumps, rng, box)
    pos = np.concatenate([bg, cl], axis=0)
    pos = np.where(pos >= box, pos - box, pos)
    return pos, np.full(n, 1.0 / n)


def lattice(nside, box=1.0, offset=0.5):
    g = (np.arange(nside) + offset) * (box / nside)
    x, y, z = np.meshgrid(g, g, g, indexing="ij")
    pos = np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)
    return pos, np.full(pos.shape[0], 1.0 / pos.shape[0])


def displaced_lattice(nside, rng, box=1.0, rms_cells=0.5):
    """Lattice plus an irrotational Gaussian displacement with |psi_k|^2 ~ k^-2,
    scaled to a 3-D rms of rms_cells mesh cells."""
    k1 = np.fft.fftfreq(nside) * nside
    kz1 = np.fft.rfftfreq(nside) * nside
    kx, ky, kz = np.meshgrid(k1, k1, kz1, indexing="ij")
    k2 = kx * kx + ky * ky + kz * kz
    k2[0, 0, 0] = 1.0
    white = np.fft.rfftn(rng.standard_normal((nside, nside, nside)))
    amp = white / k2                                   # |k psi_k / k^2| ~ k^-1 per component
    amp[0, 0, 0] = 0.0
    disp = np.stack([np.fft.irfftn(1j * kk * amp, s=(nside,) * 3) for kk in (kx, ky, kz)], axis=-1)
    disp = disp.reshape(-1, 3)
    disp *= rms_cells * (box / nside) / np.sqrt((disp ** 2).sum(axis=1).mean())
    pos, m = lattice(nside, box)
    return np.mod(pos + disp, box), m


# --- workload table -----------------------------------------------------------

def _split(mesh, box=1.0):
    rs = 1.25 * box / mesh
    return rs, 4.5 * rs


CONFIGS = {
    "uniform": dict(n=32 ** 3, mesh=32, p=4, theta=0.5, precision=0, kind="uniform"),
    "clustered": dict(n=128 ** 3, mesh=128, p=6, theta=0.5, precision=1, kind="clustered", clumps=2000),
    "batched": dict(nbox=64, mesh=64, p=5, theta=0.6, precision=1, kind="batched"),
    "large": dict(n=256 ** 3, mesh=256, p=8, theta=0.5, precision=1, kind="clustered", clumps=8000),
    "full": dict(n=512 ** 3, mesh=512, p=8, theta=0.5, precision=1, kind="full", clumps=32000),
}
# Seeds: workload k (1 .. 5, in the order above) draws from default_rng([2006_14952, k]);
# box b of the batched workload from default_rng([2006_14952, 3, b]), its sizes from
# default_rng([2006_14952, 3]).
CONFIG_INDEX = {"uniform": 1, "clustered": 2, "batched": 3, "large": 4, "full": 5}


def split_params(name):
    c = CONFIGS[name]
    rs, rcut = _split(c["mesh"])
    return dict(box=1.0, rs=rs, rcut=rcut, p=c["p"], theta=c["theta"], precision=c["precision"])


def make(name, n=None, seed_extra=()):
    """Positions and masses of a workload; ``n`` overrides the size (same recipe)."""
    c = CONFIGS[name]
    rng = rng_for(CONFIG_INDEX[name], *seed_extra)
    if c["kind"] == "uniform":
        return uniform(n or c["n"], rng)
    if c["kind"] == "clustered":
        nn = n or c["n"]
        nclump = max(1, int(round(c["clumps"] * nn / c["n"])))
        return clustered(nn, nclump, rng)
    if c["kind"] == "full":
        nside = int(round((n or c["n"]) ** (1.0 / 3.0)))
        pos, m = displaced_lattice(nside, rng)
        sub = rng.random(pos.shape[0]) < 0.5
        nclump = max(1, int(round(c["clumps"] * pos.shape[0] / c["n"])))
        pos[sub] = hernquist_clumps(int(sub.sum()), nclump, rng)
        return pos, m
    raise ValueError(name)


def batched_sizes(nbox=64, lo=12, hi=18):
    rng = rng_for(CONFIG_INDEX["batched"])
    return np.round(2.0 ** rng.uniform(lo, hi, nbox)).astype(np.int64)


def batched_box(b, n_b):
    """Box b of the batched workload: the clustered mix with round(2000 N_b / 2^21) clumps."""
    rng = rng_for(CONFIG_INDEX["batched"], b)
    nclump = max(1, int(round(2000 * n_b / 2 ** 21)))
    return clustered(int(n_b), nclump, rng)
