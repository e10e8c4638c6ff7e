"""CPU references for the long-range step (test infrastructure only).

* ``pm_forces``: the particle-mesh step written plainly with numpy FFTs, in the order of
  the method: mass deposit on a cell-centred mesh (CIC, or the higher-order TSC and PCS
  B-spline schemes), Poisson Green function filtered by exp(-k^2 r_s^2) (the Gaussian
  split of Sec. 2.2, k_s = 1/(2 r_s)), assignment window divided out twice, spectral
  gradient, inverse transforms, interpolation with the same weights.
* ``ewald_reciprocal`` / ``ewald_total``: textbook Ewald summation with splitting
  parameter alpha = 1/(2 r_s).  The real-space part is the erfc-truncated pair force of
  the short range (Sec. 2.2 force law) summed over images without a cutoff; the
  reciprocal part is the k-space sum of the same filtered Green function.  The total
  does not depend on r_s, which the tests use as a pin.
"""
from __future__ import annotations

import numpy as np

from . import bruteforce, make_params


def assignment(pos, box, M, order=2):
    """Mass-assignment weights of the B-spline schemes on a cell-centred mesh (node i at
    (i + 1/2) box/M): order 2 cloud-in-cell, 3 triangular-shaped cloud, 4 piecewise cubic.
    Returns the first node index per axis (mod M, shape (N, 3)) and the weights of the
    `order` consecutive nodes from it (shape (N, 3, order))."""
    g = np.mod(pos, box) * (M / box) - 0.5
    if order == 2:
        f = np.floor(g)
        t = g - f
        w = np.stack([1.0 - t, t], -1)
        first = f
    elif order == 3:
        c = np.floor(g + 0.5)          # nearest node
        dx = g - c                     # in [-1/2, 1/2)
        w = np.stack([0.5 * (0.5 - dx) ** 2, 0.75 - dx ** 2, 0.5 * (0.5 + dx) ** 2], -1)
        first = c - 1
    elif order == 4:
        f = np.floor(g)
        t = g - f
        w = np.stack([(1 - t) ** 3 / 6, (4 - 6 * t ** 2 + 3 * t ** 3) / 6, (1 + 3 * t + 3 * t ** 2 - 3 * t ** 3) / 6,
                      t ** 3 / 6], -1)
        first = f - 1
    else:
        raise ValueError("assignment order must be 2, 3 or 4")
    return np.mod(first.astype(np.int64), M), w


def long_range_window(k, rs=None, split=0, rcut=None):
    """Fourier factor of the long-range Green function: exp(-k^2 r_s^2) for the Gaussian
    split; for the polynomial split the transform of its smoothing density
    15/(8 pi r_c^3) (1 - r^2/r_c^2) (r < r_c), 15 (3 sin u - 3 u cos u - u^2 sin u)/u^5
    with u = k r_c (a series below u = 0.1)."""
    k = np.asarray(k, np.float64)
    if split == 0:
        return np.exp(-k * k * rs * rs)
    u = k * rcut
    out = np.empty_like(u)
    small = u < 0.1
    us = u[small]
    out[small] = 1.0 - us ** 2 / 14.0 + us ** 4 / 504.0 - us ** 6 / 33264.0
    ul = u[~small]
    out[~small] = 15.0 * (3 * np.sin(ul) - 3 * ul * np.cos(ul) - ul ** 2 * np.sin(ul)) / ul ** 5
    return out


def pm_forces(pos, mass, box, rs, M, G=1.0, split=0, rcut=None, order=2):
    """order: mass assignment (2 CIC, 3 TSC, 4 PCS); its window sinc^order per axis is
    divided out once for the deposit and once for the interpolation."""
    pos = np.asarray(pos, np.float64).reshape(-1, 3)
    i0, w = assignment(pos, box, M, order)
    d = box / M
    rho = np.zeros((M, M, M))
    stencil = [(a, b, c) for a in range(order) for b in range(order) for c in range(order)]
    for sx, sy, sz in stencil:
        wt = w[:, 0, sx] * w[:, 1, sy] * w[:, 2, sz]
        np.add.at(rho, ((i0[:, 0] + sx) % M, (i0[:, 1] + sy) % M, (i0[:, 2] + sz) % M), mass * wt / d ** 3)
    rk = np.fft.rfftn(rho)
    n1 = np.fft.fftfreq(M, 1.0 / M)
    nz = np.arange(M // 2 + 1)
    kx, ky, kz = np.meshgrid(n1 * 2 * np.pi / box, n1 * 2 * np.pi / box, nz * 2 * np.pi / box, indexing="ij")
    k2 = kx ** 2 + ky ** 2 + kz ** 2
    W = (np.sinc(kx * d / (2 * np.pi)) * np.sinc(ky * d / (2 * np.pi)) * np.sinc(kz * d / (2 * np.pi))) ** order
    nyq = np.zeros_like(k2, dtype=bool)
    if M % 2 == 0:
        nx_i, ny_i = np.meshgrid(n1, n1, indexing="ij")
        nyq |= (np.abs(nx_i) == M // 2)[:, :, None] | (np.abs(ny_i) == M // 2)[:, :, None]
        nyq[:, :, M // 2] = True
    with np.errstate(divide="ignore", invalid="ignore"):
        phi = -4 * np.pi * G * long_range_window(np.sqrt(k2), rs, split, rcut) / (k2 * W * W)
    phi[0, 0, 0] = 0.0
    phi[nyq] = 0.0
    out = np.zeros_like(pos)
    for a, ka in enumerate((kx, ky, kz)):
        am = np.fft.irfftn(-1j * ka * phi * rk, s=(M, M, M), axes=(0, 1, 2))
        g = np.zeros(len(pos))
        for sx, sy, sz in stencil:
            wt = w[:, 0, sx] * w[:, 1, sy] * w[:, 2, sz]
            g += wt * am[(i0[:, 0] + sx) % M, (i0[:, 1] + sy) % M, (i0[:, 2] + sz) % M]
        out[:, a] = g
    return out


def ewald_reciprocal(pos, mass, box, rs, G=1.0, tol=1e-16, batch=2048):
    """a_i = -G (4 pi / V) sum_{k != 0} exp(-k^2 r_s^2)/k^2 k Im(e^{i k x_i} conj(S(k))),
    S(k) = sum_j m_j e^{i k x_j}; k over the lattice 2 pi n / L up to exp(-k^2 r_s^2) < tol."""
    pos = np.asarray(pos, np.float64).reshape(-1, 3)
    kcut = np.sqrt(-np.log(tol)) / rs
    nmax = int(np.ceil(kcut * box / (2 * np.pi)))
    r = np.arange(-nmax, nmax + 1)
    n = np.stack(np.meshgrid(r, r, r, indexing="ij"), -1).reshape(-1, 3)
    # half space: each +-k pair once (the summand is even in k), doubled below
    keep = (n[:, 0] > 0) | ((n[:, 0] == 0) & (n[:, 1] > 0)) | ((n[:, 0] == 0) & (n[:, 1] == 0) & (n[:, 2] > 0))
    n = n[keep]
    k = n * (2 * np.pi / box)
    k2 = (k ** 2).sum(1)
    sel = k2 <= kcut * kcut
    k, k2 = k[sel], k2[sel]
    coef = 2.0 * (-G) * 4 * np.pi / box ** 3 * np.exp(-k2 * rs * rs) / k2
    acc = np.zeros_like(pos)
    for b in range(0, len(k), batch):
        kb = k[b:b + batch]
        ph = pos @ kb.T                           # (N, K)
        c, s = np.cos(ph), np.sin(ph)
        Sc = mass @ c                             # Re S(k)
        Ss = mass @ s                             # Im S(k)
        im = s * Sc - c * Ss                      # Im(e^{i k x_i} conj(S))
        acc += (im * coef[b:b + batch]) @ kb
    return acc


def ewald_total(pos, mass, box, rs, G=1.0):
    """Newtonian periodic acceleration (mean density removed): erfc real-space sum over
    images out to 12 r_s (must stay below box/2) plus the reciprocal sum."""
    re = 12.0 * rs
    if not re < 0.5 * box:
        raise ValueError("r_s too large for a minimum-image real-space sum")
    P = make_params(box=box, rs=rs, rcut=re, G=G)
    return bruteforce(pos, mass, P, rc=re) + ewald_reciprocal(pos, mass, box, rs, G)
