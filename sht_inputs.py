"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module holds no transform arithmetic: it only builds grid geometries
(ring colatitudes, pixel counts, azimuth offsets, quadrature weights) and
draws random coefficient sets and maps.  Both the CPU reference in
``oracle/`` and the GPU library consume what it returns.

Grids
-----
* Gauss-Legendre: ``nrings`` rings at the roots of P_nrings(cos theta), equal
  pixel counts.  Weights follow Eq. 2 of the paper: w_y includes the
  2 pi / Nphi_y factor, i.e. w_y = w_GL,y * 2 pi / Nphi_y.  South rings are
  built as pi - theta_north so that ring pairs are exact mirrors.
* HEALPix (Gorski et al. 2005) ring scheme: 4 Nside - 1 rings; polar caps with
  4i pixels, the equatorial belt with 4 Nside pixels; uniform weights
  4 pi / Npix (no iteration).

Coefficients
------------
a_lm with E|a_lm|^2 = C_l: for m > 0 Re and Im are N(0, C_l/2), for m = 0 the
coefficient is real N(0, C_l).  ``powerlaw`` uses C_l = 1/(l+1)^2; ``unit``
draws Re and Im from N(0, 1) (Im = 0 at m = 0).  Spin-2 sets are zero for
l < 2.  Seeds: numpy ``default_rng([13034945, tag, transform, component])``.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

SEED_ROOT = 13034945


@dataclasses.dataclass
class Geometry:
    theta: np.ndarray          # float64 [nrings]
    nphi: np.ndarray           # int64 [nrings]
    phi0: np.ndarray           # float64 [nrings]
    weight: np.ndarray         # float64 [nrings], includes 2 pi / nphi
    ofs: np.ndarray            # int64 [nrings], first pixel of each ring
    stride: int = 1

    @property
    def nrings(self) -> int:
        return int(self.theta.shape[0])

    @property
    def npix(self) -> int:
        return int(np.max(self.ofs + (self.nphi - 1) * self.stride) + 1)

    def subset(self, rings) -> "Geometry":
        """Geometry restricted to the given ring indices (pixel offsets kept)."""
        rings = np.asarray(rings, dtype=np.int64)
        return Geometry(self.theta[rings].copy(), self.nphi[rings].copy(),
                        self.phi0[rings].copy(), self.weight[rings].copy(),
                        self.ofs[rings].copy(), self.stride)


def _packed_offsets(nphi: np.ndarray) -> np.ndarray:
    ofs = np.zeros_like(nphi)
    ofs[1:] = np.cumsum(nphi)[:-1]
    return ofs


def _gauss_legendre_theta(n: int):
    """Gauss-Legendre nodes as colatitudes (ascending) and their weights, by
    Newton's method on P_n(cos theta) in long double (numpy's leggauss loses
    ~1e-14 in the weights at n ~ 100, enough to spoil a 1e-12 round trip)."""
    ld = np.longdouble
    k = np.arange(1, n + 1).astype(ld)
    th = (ld(np.pi) * (4 * k - 1) / (4 * n + 2)).astype(ld)

    def legendre(c):
        p0 = np.ones_like(c)
        p1 = c.copy()
        for j in range(2, n + 1):
            p0, p1 = p1, ((2 * j - 1) * c * p1 - (j - 1) * p0) / j
        if n == 1:
            p0, p1 = np.ones_like(c), c
        dp = n * (c * p1 - p0) / (c * c - 1)
        return p1, dp

    for _ in range(12):
        c = np.cos(th)
        p, dp = legendre(c)
        step = p / (-np.sin(th) * dp)
        th = th - step
        if np.max(np.abs(step)) < 1e-17:     # quadratic convergence: done
            break
    c = np.cos(th)
    _, dp = legendre(c)
    w = 2 / ((1 - c * c) * dp * dp)
    return th, w


def gauss_geometry(nrings: int, nphi: int, phi0: float = 0.0) -> Geometry:
    """Gauss-Legendre rings ordered north to south."""
    thl, wl = _gauss_legendre_theta(nrings)
    order = np.argsort(thl)
    theta = thl[order].astype(np.float64)
    w = wl[order].astype(np.float64)
    nh = nrings // 2
    # exact mirror pairs: south = pi - north; symmetric weights
    for i in range(nh):
        j = nrings - 1 - i
        theta[j] = math.pi - theta[i]
        w[j] = w[i]
    if nrings % 2 == 1:
        theta[nh] = 0.5 * math.pi
    nph = np.full(nrings, nphi, dtype=np.int64)
    weight = w * (2.0 * math.pi / nph)
    return Geometry(theta, nph, np.full(nrings, float(phi0)), weight,
                    _packed_offsets(nph))


def mixed_geometry(nphi_north, phi0: float = 0.0) -> Geometry:
    """Gauss-Legendre colatitudes for 2 * len(nphi_north) rings with per-ring
    pixel counts: ring i of the north half and its southern mirror both get
    nphi_north[i] pixels (so that FFT lengths of every kind can be mixed in
    one grid).  phi0 grows by phi0 per ring."""
    nh = len(nphi_north)
    g = gauss_geometry(2 * nh, 1)
    nph = np.asarray(list(nphi_north) + list(nphi_north)[::-1], dtype=np.int64)
    wgl = g.weight * (2.0 * math.pi) ** -1       # back to the GL weights (nphi = 1)
    weight = wgl * (2.0 * math.pi / nph)
    ph = phi0 * np.arange(2 * nh, dtype=np.float64)
    return Geometry(g.theta, nph, ph, weight, _packed_offsets(nph))


ECP_FEJER1, ECP_FEJER2, ECP_CC = 0, 1, 2


def ecp_rule(n: int, kind: int):
    """Colatitudes (north to south) and weights on [-1, 1] in x = cos theta of
    the equidistant rules: Fejer's first rule (theta = (k + 1/2) pi / n),
    Fejer's second rule (theta = k pi / (n + 1), k = 1 .. n) and Clenshaw-Curtis
    (theta = k pi / (n - 1), k = 0 .. n - 1), from their closed-form sums."""
    if kind == ECP_FEJER1:
        th = np.pi * (np.arange(n) + 0.5) / n
        j = np.arange(1, n // 2 + 1)
        w = (2.0 / n) * (1.0 - 2.0 * (np.cos(2.0 * np.outer(th, j)) / (4.0 * j * j - 1.0)).sum(axis=1))
    elif kind == ECP_FEJER2:
        th = np.pi * np.arange(1, n + 1) / (n + 1)
        j = np.arange(1, (n + 1) // 2 + 1)
        w = 4.0 * np.sin(th) / (n + 1) * (np.sin(np.outer(th, 2 * j - 1)) / (2 * j - 1)).sum(axis=1)
    elif kind == ECP_CC:
        N = n - 1
        th = np.pi * np.arange(n) / N
        j = np.arange(1, N // 2 + 1)
        b = np.where(2 * j == N, 1.0, 2.0)
        c = np.where((np.arange(n) == 0) | (np.arange(n) == N), 1.0, 2.0)
        w = c / N * (1.0 - (b * np.cos(2.0 * np.outer(th, j)) / (4.0 * j * j - 1.0)).sum(axis=1))
    else:
        raise ValueError(kind)
    return th, w


def ecp_geometry(nrings: int, nphi: int, kind: int, phi0: float = 0.0) -> Geometry:
    """Equidistant-cylindrical grid with the rule of `kind` (weights times 2 pi / nphi)."""
    th, w = ecp_rule(nrings, kind)
    nph = np.full(nrings, nphi, dtype=np.int64)
    return Geometry(th, nph, np.full(nrings, float(phi0)), w * (2.0 * math.pi / nph),
                    _packed_offsets(nph))


def _smooth235(n: int) -> bool:
    for p in (2, 3, 5):
        while n % p == 0:
            n //= p
    return n == 1


def reduced_gauss_geometry(nrings: int, nphi_max: int, lmax: int, mmax: int, spin: int,
                           phi0: float = 0.0) -> Geometry:
    """Gauss-Legendre rings, ring y with 2 m_y + 1 pixels rounded up to the next
    2,3,5-smooth number (at most nphi_max), m_y <= mmax the largest m whose terms
    the polar criterion sqrt(m^2 + s^2 - 2 m s |cos t|) - lmax sin t <= T keeps,
    T = max(100, lmax / 100)."""
    g = gauss_geometry(nrings, 1, phi0)
    wgl = g.weight / (2.0 * math.pi)
    T = max(100.0, 0.01 * lmax)
    nph = np.zeros(nrings, dtype=np.int64)
    for y in range(nrings):
        c, st = abs(math.cos(g.theta[y])), math.sin(g.theta[y])
        m = mmax
        while m > 0 and math.sqrt(max(0.0, m * m + spin * spin - 2.0 * m * spin * c)) - lmax * st > T:
            m -= 1
        n = 2 * m + 1
        while not _smooth235(n):
            n += 1
        nph[y] = min(n, nphi_max)
    return Geometry(g.theta, nph, g.phi0, wgl * (2.0 * math.pi / nph), _packed_offsets(nph))


def healpix_geometry(nside: int) -> Geometry:
    """HEALPix ring-scheme geometry (pixel order within a ring as in HEALPix)."""
    nr = 4 * nside - 1
    theta = np.zeros(nr)
    nph = np.zeros(nr, dtype=np.int64)
    phi0 = np.zeros(nr)
    for i in range(1, 2 * nside + 1):           # north cap + north belt + equator
        y = i - 1
        if i < nside:
            theta[y] = 2.0 * math.asin(i / (math.sqrt(6.0) * nside))
            nph[y] = 4 * i
            phi0[y] = math.pi / (4.0 * i)
        else:
            z = (4.0 / 3.0) - 2.0 * i / (3.0 * nside)
            theta[y] = math.acos(z)
            nph[y] = 4 * nside
            s = (i - nside + 1) % 2
            phi0[y] = (math.pi / (2.0 * nside)) * (1.0 - 0.5 * s)
    for y in range(2 * nside, nr):              # south: mirrors of the north
        yn = nr - 1 - y
        theta[y] = math.pi - theta[yn]
        nph[y] = nph[yn]
        phi0[y] = phi0[yn]
    theta[2 * nside - 1] = 0.5 * math.pi
    npix = 12 * nside * nside
    weight = np.full(nr, 4.0 * math.pi / npix)
    return Geometry(theta, nph, phi0, weight, _packed_offsets(nph))


def nalm(lmax: int, mmax: int) -> int:
    return (mmax + 1) * (lmax + 1) - (mmax * (mmax + 1)) // 2


def alm_index(lmax: int, l, m):
    return m * (2 * lmax + 1 - m) // 2 + l


def lm_arrays(lmax: int, mmax: int):
    """(l, m) of every stored coefficient, in storage order."""
    ls, ms = [], []
    for m in range(mmax + 1):
        ls.append(np.arange(m, lmax + 1))
        ms.append(np.full(lmax + 1 - m, m))
    return np.concatenate(ls), np.concatenate(ms)


def random_alm(lmax: int, mmax: int, ntrans: int = 1, spin: int = 0,
               spectrum: str = "powerlaw", tag: int = 0) -> np.ndarray:
    """Complex coefficient sets as float64 [ntrans][ncomp][nalm][2]."""
    ncomp = 2 if spin else 1
    ls, ms = lm_arrays(lmax, mmax)
    n = ls.shape[0]
    if spectrum == "uniform":
        # Re and Im uniform on [-1, 1), Im a_l0 = 0 (the accuracy tests' coefficients)
        out = np.empty((ntrans, ncomp, n, 2))
        for t in range(ntrans):
            for c in range(ncomp):
                rng = np.random.default_rng([SEED_ROOT, tag, t, c])
                out[t, c] = rng.uniform(-1.0, 1.0, (n, 2))
        out[..., 1] = np.where(ms == 0, 0.0, out[..., 1])
        if spin:
            out[:, :, ls < spin, :] = 0.0
        return out
    if spectrum == "unit":
        sd_re = np.ones(n)
        sd_im = np.where(ms == 0, 0.0, 1.0)
    elif spectrum == "powerlaw":
        cl = 1.0 / (ls + 1.0) ** 2
        sd_re = np.where(ms == 0, np.sqrt(cl), np.sqrt(cl / 2.0))
        sd_im = np.where(ms == 0, 0.0, np.sqrt(cl / 2.0))
    else:
        raise ValueError(spectrum)
    if spin:
        sd_re = np.where(ls < spin, 0.0, sd_re)
        sd_im = np.where(ls < spin, 0.0, sd_im)
    out = np.empty((ntrans, ncomp, n, 2))
    for t in range(ntrans):
        for c in range(ncomp):
            rng = np.random.default_rng([SEED_ROOT, tag, t, c])
            out[t, c, :, 0] = rng.standard_normal(n)
            out[t, c, :, 1] = rng.standard_normal(n)
            out[t, c, :, 0] *= sd_re
            out[t, c, :, 1] *= sd_im
    return out


def random_map(geom: Geometry, ntrans: int = 1, ncomp: int = 1, sigma: float = 1.0,
               tag: int = 0) -> np.ndarray:
    """White-noise maps float64 [ntrans][ncomp][npix]."""
    out = np.zeros((ntrans, ncomp, geom.npix))
    for t in range(ntrans):
        for c in range(ncomp):
            rng = np.random.default_rng([SEED_ROOT, 1000 + tag, t, c])
            out[t, c] = sigma * rng.standard_normal(geom.npix)
    return out


# The five workloads: (name, geometry builder, lmax, spin, ntrans)
WORKLOADS = {
    "gl127": dict(desc="GL 128 rings x 255 px, lmax=mmax=127, spin 0, 1 transform, "
                       "Re/Im ~ N(0,1)", grid=("gauss", 128, 255), lmax=127, spin=0,
                  ntrans=1, spectrum="unit"),
    "hp1024": dict(desc="HEALPix Nside=1024, lmax=mmax=2047, spin 0, 1 transform, "
                        "C_l=1/(l+1)^2", grid=("healpix", 1024), lmax=2047, spin=0,
                   ntrans=1, spectrum="powerlaw"),
    "gl4095s2": dict(desc="GL 4096 rings x 8191 px, lmax=mmax=4095, spin 2 (E/B<->Q/U), "
                          "16 transforms, C_l=1/(l+1)^2", grid=("gauss", 4096, 8191),
                     lmax=4095, spin=2, ntrans=16, spectrum="powerlaw"),
    "hp2048": dict(desc="HEALPix Nside=2048, lmax=mmax=4095, spin 0, 8 maps",
                   grid=("healpix", 2048), lmax=4095, spin=0, ntrans=8,
                   spectrum="powerlaw"),
}


def make_geometry(grid) -> Geometry:
    if grid[0] == "gauss":
        return gauss_geometry(grid[1], grid[2])
    if grid[0] == "healpix":
        return healpix_geometry(grid[1])
    raise ValueError(grid)


def mixed_batch_lmaxes():
    """The mixed batch: 16 transforms each at lmax 255, 511, 1023, 2047 on
    Gauss-Legendre grids with lmax+1 rings and 2 lmax + 1 pixels per ring."""
    return [255, 511, 1023, 2047]
