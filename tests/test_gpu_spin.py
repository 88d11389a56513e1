"""Spin transforms for spins other than 0 and 2 (Sect. 4.1: the recursion of
Eq. 11 for any s), including odd spins, where real Q and U give
Q - iU = (-1)^s sum -s_a -s_Y, and s = 37, the spin of the paper's tests."""
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


CASES = {
    # name: (geometry, lmax, mmax, spin, ntrans)
    "gl_s1": (lambda: si.gauss_geometry(32, 63, 0.2), 31, 31, 1, 2),
    "gl_s3_mmax": (lambda: si.gauss_geometry(30, 61, 0.1), 29, 20, 3, 3),
    "gl_s4": (lambda: si.gauss_geometry(24, 49), 23, 23, 4, 1),
    "gl_s37": (lambda: si.gauss_geometry(64, 129, 0.3), 63, 63, 37, 2),
    "hp_s1_alias": (lambda: si.healpix_geometry(8), 22, 22, 1, 2),
    "unpaired_s5": (lambda: si.ecp_geometry(17, 41, si.ECP_FEJER1, 0.4), 20, 18, 5, 1),
}


def _setup(name, precision="fp64"):
    sht = _sht()
    build, lmax, mmax, spin, ntrans = CASES[name]
    g = build()
    plan = sht.Plan(sht.Geometry.from_inputs(g), lmax, mmax, spin=spin, ntrans=ntrans, precision=precision)
    a = si.random_alm(lmax, mmax, ntrans, spin, tag=500 + spin)
    return g, plan, a


@pytest.mark.parametrize("name", sorted(CASES))
def test_spin_parity(name):
    g, plan, a = _setup(name)
    _, lmax, mmax, spin, _ = CASES[name]
    mp = to_host(plan.alm2map(to_dev(a)))
    assert rel_err(mp, oracle.synthesis(g, lmax, mmax, spin, a)) < TOL64
    back = to_host(plan.map2alm(to_dev(mp)))
    assert rel_err(back, oracle.analysis(g, lmax, mmax, spin, mp)) < TOL64
    if name.startswith("gl_"):            # exact quadrature: the round trip returns a
        assert rel_err(back, a) < 1e-11


@pytest.mark.parametrize("name", ["gl_s1", "gl_s37"])
def test_spin_adjoint_identity(name):
    """<Y a, x> = sum over l, m >= 0 of fac_m Re(a_lm conj((Y^T x)_lm))."""
    g, plan, a = _setup(name)
    _, lmax, mmax, spin, ntrans = CASES[name]
    x = si.random_map(g, ntrans, 2, tag=510)
    ya = to_host(plan.alm2map(to_dev(a)))
    yt = to_host(plan.adjoint(to_dev(x)))
    _, ms = si.lm_arrays(lmax, mmax)
    fac = np.where(ms == 0, 1.0, 2.0)
    lhs = float(np.sum(ya * x))
    rhs = float(np.sum(fac[None, None, :] * (a[..., 0] * yt[..., 0] + a[..., 1] * yt[..., 1])))
    assert abs(lhs - rhs) <= 1e-12 * np.sqrt(np.sum(ya * ya) * np.sum(x * x))


def test_spin3_fp32_mfma_form():
    g, plan, a = _setup("gl_s3_mmax", precision="fp32_mfma")
    mp = to_host(plan.alm2map(to_dev(a)))
    assert rel_err(mp, oracle.synthesis(g, 29, 20, 3, a)) < 1e-6


def test_spin1_batch_equals_plans():
    sht = _sht()
    plans, alms = [], []
    for k, lmax in enumerate([15, 31]):
        g = si.gauss_geometry(lmax + 1, 2 * lmax + 1, 0.1 * k)
        plans.append(sht.Plan(sht.Geometry.from_inputs(g), lmax, spin=1, ntrans=2))
        alms.append(to_dev(si.random_alm(lmax, lmax, 2, 1, tag=520 + k)))
    b = sht.Batch(plans)
    maps = b.alm2map(alms)
    for p, a, mp in zip(plans, alms, maps):
        assert np.array_equal(to_host(mp), to_host(p.alm2map(a)))
    backs = b.map2alm(maps)
    for p, mp, bk in zip(plans, maps, backs):
        assert np.array_equal(to_host(bk), to_host(p.map2alm(mp)))
