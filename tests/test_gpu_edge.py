"""Degenerate and ragged cases against the oracle on the GPU.

* the smallest transforms: lmax 0 on one ring of one pixel; lmax = spin = 2;
* mmax = 0 (only the axisymmetric part) for spin 0 and 2;
* rings without a mirror (every slot unpaired) with irregular pixel counts,
  weights and azimuth offsets;
* transform counts that leave the last column group partly empty;
* a strided pixel layout (pixels of a ring `stride` apart, rings at arbitrary
  offsets); pixels outside the rings are not written.
"""
import math

import numpy as np
import pytest

import oracle
import sht_inputs as si
from gpu_util import rel_err, to_dev, to_host

pytestmark = pytest.mark.gpu

TOL64 = 1e-11


def _sht():
    import paper_1303_4945_amd as sht
    return sht


def _ring_pixels(g):
    return np.concatenate([g.ofs[y] + np.arange(g.nphi[y]) * g.stride for y in range(g.nrings)])


def _check(g, lmax, mmax, spin, ntrans, tag):
    sht = _sht()
    geom = sht.Geometry.from_inputs(g)
    plan = sht.Plan(geom, lmax, mmax, spin=spin, ntrans=ntrans)
    a = si.random_alm(lmax, mmax, ntrans, spin, tag=tag)
    mp = to_host(plan.alm2map(to_dev(a)))
    ref = oracle.synthesis(g, lmax, mmax, spin, a)
    pix = _ring_pixels(g)
    assert rel_err(mp[..., pix], ref[..., pix]) < TOL64
    # analysis of an oracle-made map (zeros between the rings)
    back = to_host(plan.map2alm(to_dev(ref)))
    ref_a = oracle.analysis(g, lmax, mmax, spin, ref)
    assert rel_err(back, ref_a) < TOL64
    adj = to_host(plan.adjoint(to_dev(ref)))
    assert rel_err(adj, oracle.adjoint_synthesis(g, lmax, mmax, spin, ref)) < TOL64


def test_lmax0_one_pixel():
    _check(si.gauss_geometry(1, 1), 0, 0, 0, 1, tag=201)


def test_lmax_equals_spin():
    _check(si.gauss_geometry(3, 5, 0.2), 2, 2, 2, 1, tag=202)


@pytest.mark.parametrize("spin", [0, 2])
def test_mmax0(spin):
    _check(si.gauss_geometry(18, 35, 0.4), 17, 0, spin, 2, tag=203 + spin)


@pytest.mark.parametrize("spin", [0, 2])
def test_unpaired_irregular_rings(spin):
    theta = np.array([0.05, 0.3, 1.1, 0.5 * math.pi, 2.0, 2.9])
    nphi = np.array([3, 7, 12, 9, 10, 5], dtype=np.int64)
    phi0 = np.array([0.0, 0.4, 1.3, 0.2, 2.5, 0.9])
    weight = np.array([0.02, 0.1, 0.3, 0.35, 0.25, 0.07])
    ofs = np.concatenate([[0], np.cumsum(nphi)[:-1]]).astype(np.int64)
    g = si.Geometry(theta, nphi, phi0, weight, ofs, 1)
    _check(g, 6, 5, spin, 3, tag=210 + spin)


@pytest.mark.parametrize("spin,ntrans", [(2, 9), (0, 17)])
def test_ragged_transform_groups(spin, ntrans):
    _check(si.gauss_geometry(20, 39, 0.1), 19, 19, spin, ntrans, tag=220 + spin)


def test_strided_pixels():
    g0 = si.gauss_geometry(10, 19, 0.3)
    stride = 3
    ofs = (np.arange(g0.nrings, dtype=np.int64) * (19 * stride + 5) + 2)
    g = si.Geometry(g0.theta, g0.nphi, g0.phi0, g0.weight, ofs, stride)
    _check(g, 9, 9, 2, 2, tag=230)
