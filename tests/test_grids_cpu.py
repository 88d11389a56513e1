"""ECP grids (Fejer's first and second rules, Clenshaw-Curtis) and the reduced
Gauss-Legendre grid (Sect. 4.4): the library's constructors against the
independent constructions of the test inputs, and the quadrature rules
against Legendre polynomials (host only, no GPU)."""
import math

import numpy as np
import numpy.polynomial.legendre as npl
import pytest

import sht_inputs as si


def _sht():
    import paper_1303_4945_amd as sht
    return sht


@pytest.mark.parametrize("kind", [si.ECP_FEJER1, si.ECP_FEJER2, si.ECP_CC])
@pytest.mark.parametrize("n", [2, 3, 8, 33, 256])
def test_ecp_rules_integrate_legendre_polynomials(kind, n):
    """sum_k w_k P_j(x_k) = 2 delta_j0 for every degree j <= n - 1."""
    th, w = si.ecp_rule(n, kind)
    assert np.all(np.diff(th) > 0) and th[0] >= 0 and th[-1] <= math.pi
    x = np.cos(th)
    for j in range(n):
        c = np.zeros(j + 1)
        c[j] = 1.0
        assert abs(np.sum(w * npl.legval(x, c)) - (2.0 if j == 0 else 0.0)) < 1e-13


def test_ecp_node_sets():
    th, _ = si.ecp_rule(4, si.ECP_FEJER1)
    assert np.allclose(th, np.pi * np.array([0.5, 1.5, 2.5, 3.5]) / 4)
    th, _ = si.ecp_rule(3, si.ECP_FEJER2)
    assert np.allclose(th, np.pi * np.array([1, 2, 3]) / 4)
    th, w = si.ecp_rule(3, si.ECP_CC)
    assert np.allclose(th, [0.0, 0.5 * np.pi, np.pi])
    assert np.allclose(w, [1 / 3, 4 / 3, 1 / 3])          # Simpson's rule


@pytest.mark.parametrize("kind", [si.ECP_FEJER1, si.ECP_FEJER2, si.ECP_CC])
@pytest.mark.parametrize("n", [2, 7, 64, 1025])
def test_ecp_geometry_matches_inputs(kind, n):
    sht = _sht()
    r = sht.Geometry.ecp(n, 2 * n + 3, kind, 0.3).rings()
    ref = si.ecp_geometry(n, 2 * n + 3, kind, 0.3)
    assert np.max(np.abs(r["theta"] - ref.theta)) < 4e-15
    assert np.max(np.abs(r["weight"] - ref.weight)) < 1e-14 * np.max(ref.weight)
    assert np.array_equal(r["nphi"], ref.nphi) and np.array_equal(r["ofs"], ref.ofs)
    assert np.allclose(r["phi0"], 0.3)


@pytest.mark.parametrize("lmax,spin", [(255, 0), (255, 2), (1023, 0), (2047, 2)])
def test_reduced_gauss_matches_inputs(lmax, spin):
    sht = _sht()
    nr, nmax = lmax + 1, 2 * lmax + 2
    r = sht.Geometry.reduced_gauss(nr, nmax, lmax, lmax, spin, 0.1).rings()
    ref = si.reduced_gauss_geometry(nr, nmax, lmax, lmax, spin, 0.1)
    assert np.array_equal(r["nphi"], ref.nphi)
    assert np.max(np.abs(r["theta"] - ref.theta)) < 4e-15
    # (two independent Gauss-Legendre weight computations: ~1e-13 at the polar
    # rings of a 2048-ring grid)
    assert np.max(np.abs(r["weight"] / ref.weight - 1)) < 5e-13
    # every ring length is 2,3,5-smooth (or the cap), the grid keeps the
    # mirror symmetry, and the quadrature still integrates 1 over the sphere
    for n in r["nphi"]:
        k = int(n)
        for p in (2, 3, 5):
            while k % p == 0:
                k //= p
        assert k == 1 or n == nmax
    assert np.array_equal(r["nphi"], r["nphi"][::-1])
    assert abs(np.sum(r["weight"] * r["nphi"]) - 4 * math.pi) < 1e-11


def test_reduced_gauss_saves_pixels():
    """The thinning removes a third of the pixels of the full grid at lmax 4095."""
    g = si.reduced_gauss_geometry(4096, 8192, 4095, 4095, 0)
    assert 1.0 - g.nphi.sum() / (4096 * 8191) > 0.30
    assert g.nphi[2048] == 8192 and g.nphi[0] < 300


@pytest.mark.parametrize("spin", [0, 2, 37])
def test_uniform_coefficients_recipe(spin):
    """The accuracy test's coefficients: Re and Im uniform on [-1, 1), Im a_l0 = 0,
    l < spin zero, seeded (two calls agree, another tag differs)."""
    lmax = 63
    a = si.random_alm(lmax, lmax, 2, spin, spectrum="uniform", tag=5)
    ls, ms = si.lm_arrays(lmax, lmax)
    assert a.shape == (2, 2 if spin else 1, ls.size, 2)
    assert np.all(a >= -1.0) and np.all(a < 1.0)
    assert np.all(a[:, :, ms == 0, 1] == 0.0)
    assert np.all(a[:, :, ls < spin, :] == 0.0)
    live = a[:, :, (ls >= spin) & (ms > 0), :]
    assert abs(live.mean()) < 0.02 and abs(live.var() - 1.0 / 3.0) < 0.02   # U(-1, 1): mean 0, variance 1/3
    assert np.array_equal(a, si.random_alm(lmax, lmax, 2, spin, spectrum="uniform", tag=5))
    assert not np.array_equal(a, si.random_alm(lmax, lmax, 2, spin, spectrum="uniform", tag=6))
