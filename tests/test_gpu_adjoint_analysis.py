"""The adjoint of analysis, W Y (Sect. 4.5): synthesis with every ring
multiplied by its weight, against the oracle, and the adjoint identity
<x, W Y a> = sum over l, m >= 0 of fac_m Re(a_lm conj((Y^T W x)_lm)) with
fac_0 = 1 and fac_m = 2 for m > 0 (real maps, coefficients stored for m >= 0)."""
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
    "gl_s0": (lambda: si.gauss_geometry(24, 47, 0.2), 23, 23, 0, 2),
    "gl_s2": (lambda: si.gauss_geometry(20, 41, 0.1), 19, 17, 2, 3),
    "hp_s0": (lambda: si.healpix_geometry(8), 20, 20, 0, 1),
    "hp_s2": (lambda: si.healpix_geometry(8), 18, 18, 2, 2),
}


def _ring_weights_per_pixel(g):
    w = np.zeros(g.npix)
    for y in range(g.nrings):
        w[g.ofs[y] + np.arange(g.nphi[y]) * g.stride] = g.weight[y]
    return w


@pytest.mark.parametrize("name", sorted(CASES))
def test_adjoint_analysis_against_oracle(name):
    sht = _sht()
    build, lmax, mmax, spin, ntrans = CASES[name]
    g = build()
    plan = sht.Plan(sht.Geometry.from_inputs(g), lmax, mmax, spin=spin, ntrans=ntrans)
    a = si.random_alm(lmax, mmax, ntrans, spin, tag=300 + len(name))
    got = to_host(plan.adjoint_analysis(to_dev(a)))
    ref = oracle.synthesis(g, lmax, mmax, spin, a) * _ring_weights_per_pixel(g)
    assert rel_err(got, ref) < TOL64
    # the stage entry point gives the same maps from the same phases
    F = plan.legendre_synth(to_dev(a))
    assert np.array_equal(to_host(plan.ring_synth(F, weights=True)), got)


@pytest.mark.parametrize("name", ["gl_s0", "gl_s2", "hp_s2"])
def test_adjoint_identity(name):
    sht = _sht()
    build, lmax, mmax, spin, ntrans = CASES[name]
    g = build()
    plan = sht.Plan(sht.Geometry.from_inputs(g), lmax, mmax, spin=spin, ntrans=ntrans)
    a = si.random_alm(lmax, mmax, ntrans, spin, spectrum="unit", tag=320)
    x = si.random_map(g, ntrans, 2 if spin else 1, tag=321)
    wya = to_host(plan.adjoint_analysis(to_dev(a)))
    ax = to_host(plan.map2alm(to_dev(x)))
    _, ms = si.lm_arrays(lmax, mmax)
    fac = np.where(ms == 0, 1.0, 2.0)
    lhs = float(np.sum(x * wya))
    rhs = float(np.sum(fac[None, None, :] * (a[..., 0] * ax[..., 0] + a[..., 1] * ax[..., 1])))
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + np.sqrt(np.sum(x * x) * np.sum(wya * wya)))
