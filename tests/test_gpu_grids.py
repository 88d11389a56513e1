"""Transforms on the ECP grids and the reduced Gauss-Legendre grid (Sect. 4.4)
against the oracle, and their round trips: exact on the ECP grids with enough
rings (the rules integrate the degree-2 lmax products exactly), accurate to
the polar criterion's precision on the reduced grid."""
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


def _run(g, lmax, spin, ntrans, tag):
    sht = _sht()
    plan = sht.Plan(sht.Geometry.from_inputs(g), lmax, spin=spin, ntrans=ntrans)
    a = si.random_alm(lmax, lmax, ntrans, spin, tag=tag)
    mp = plan.alm2map(to_dev(a))
    back = to_host(plan.map2alm(mp))
    mp = to_host(mp)
    return a, mp, back


@pytest.mark.parametrize("kind", [si.ECP_FEJER1, si.ECP_FEJER2, si.ECP_CC])
@pytest.mark.parametrize("spin", [0, 2])
def test_ecp_grids(kind, spin):
    lmax = 40
    # 2 lmax + 2 rings: the rule is exact to degree 2 lmax + 1
    g = si.ecp_geometry(2 * lmax + 2, 2 * lmax + 1, kind, 0.25)
    a, mp, back = _run(g, lmax, spin, 2, tag=400 + 10 * kind + spin)
    assert rel_err(mp, oracle.synthesis(g, lmax, lmax, spin, a)) < TOL64
    assert rel_err(back, oracle.analysis(g, lmax, lmax, spin, mp)) < TOL64
    assert rel_err(back, a) < 1e-11


@pytest.mark.parametrize("spin", [0, 2])
def test_reduced_gauss_grid(spin):
    lmax = 383
    g = si.reduced_gauss_geometry(lmax + 1, 2 * lmax + 2, lmax, lmax, spin, 0.1)
    assert g.nphi.sum() < (lmax + 1) * (2 * lmax + 1)       # thinned near the poles
    a, mp, back = _run(g, lmax, spin, 2, tag=420 + spin)
    rings = np.array([0, 1, 5, 40, lmax // 2, lmax - 1, lmax])
    ref = oracle.synthesis(g, lmax, lmax, spin, a, rings=rings)
    pix = np.concatenate([np.arange(g.ofs[y], g.ofs[y] + g.nphi[y]) for y in rings])
    assert rel_err(mp[..., pix], ref[..., pix]) < TOL64
    ms = np.array([0, 1, 2, 100, 300, lmax])
    ref_a = oracle.analysis(g, lmax, lmax, spin, mp, ms=ms)
    sel = np.concatenate([np.arange(m * (2 * lmax + 1 - m) // 2 + m, m * (2 * lmax + 1 - m) // 2 + lmax + 1)
                          for m in ms])
    assert rel_err(back[:, :, sel], ref_a[:, :, sel]) < TOL64
    # not exact in a mathematical sense, but to the precision of the criterion
    assert rel_err(back, a) < 1e-10


def test_library_grid_constructors_on_device():
    """The geometries built by the library transform like the test inputs' ones."""
    sht = _sht()
    lmax = 30
    a = to_dev(si.random_alm(lmax, lmax, 1, 0, tag=430))
    p1 = sht.Plan(sht.Geometry.ecp(2 * lmax + 2, 2 * lmax + 1, si.ECP_CC), lmax)
    p2 = sht.Plan(sht.Geometry.from_inputs(si.ecp_geometry(2 * lmax + 2, 2 * lmax + 1, si.ECP_CC)), lmax)
    assert rel_err(to_host(p1.alm2map(a)), to_host(p2.alm2map(a))) < 1e-14
    p3 = sht.Plan(sht.Geometry.reduced_gauss(lmax + 1, 2 * lmax + 2, lmax), lmax)
    assert rel_err(to_host(p3.map2alm(p3.alm2map(a))), to_host(a)) < 1e-11
