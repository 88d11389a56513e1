"""Pins for the CPU reference (oracle/), independent of the oracle's own code.

Each test checks the oracle against something the mathematics or a library
fixes: textbook closed forms, scipy/mpmath special functions, exact
invariants (addition theorem, parity, Wigner-d orthogonality), brute-force
pixel sums, Gauss-Legendre quadrature exactness, and the adjoint identity.
"""
import math

import mpmath
import numpy as np
import pytest
from scipy.special import lpmv, sph_harm_y

import oracle
import sht_inputs as si

FOURPI = 4.0 * math.pi


# ---------------------------------------------------------------- lambda, s=0
def _ylm_closed(l, m, t):
    """Textbook Condon-Shortley Y_lm(theta, 0) for 0 <= m <= l <= 4."""
    c, s = math.cos(t), math.sin(t)
    p = math.pi
    table = {
        (0, 0): 0.5 / math.sqrt(p),
        (1, 0): math.sqrt(3 / (4 * p)) * c,
        (1, 1): -math.sqrt(3 / (8 * p)) * s,
        (2, 0): math.sqrt(5 / (16 * p)) * (3 * c * c - 1),
        (2, 1): -math.sqrt(15 / (8 * p)) * s * c,
        (2, 2): math.sqrt(15 / (32 * p)) * s * s,
        (3, 0): math.sqrt(7 / (16 * p)) * (5 * c ** 3 - 3 * c),
        (3, 1): -math.sqrt(21 / (64 * p)) * s * (5 * c * c - 1),
        (3, 2): math.sqrt(105 / (32 * p)) * s * s * c,
        (3, 3): -math.sqrt(35 / (64 * p)) * s ** 3,
        (4, 0): (3 / 16) * math.sqrt(1 / p) * (35 * c ** 4 - 30 * c * c + 3),
        (4, 1): -(3 / 8) * math.sqrt(5 / p) * s * (7 * c ** 3 - 3 * c),
        (4, 2): (3 / 8) * math.sqrt(5 / (2 * p)) * s * s * (7 * c * c - 1),
        (4, 3): -(3 / 8) * math.sqrt(35 / p) * s ** 3 * c,
        (4, 4): (3 / 16) * math.sqrt(35 / (2 * p)) * s ** 4,
    }
    return table[(l, m)]


@pytest.mark.parametrize("theta", [1e-3, 0.3, 1.1, math.pi / 2, 2.0, math.pi - 1e-3])
def test_lambda_s0_closed_forms(theta):
    for m in range(0, 5):
        lam = oracle.lam(4, m, 0, theta)
        lam_neg = oracle.lam(4, -m, 0, theta)
        for l in range(m, 5):
            ref = _ylm_closed(l, m, theta)
            assert abs(lam[l] - ref) <= 2e-15 * max(1.0, abs(ref)), (l, m)
            # Condon-Shortley: Y_{l,-m}(theta, 0) = (-1)^m Y_lm(theta, 0)
            assert abs(lam_neg[l] - (-1) ** m * ref) <= 2e-15, (l, -m)


def test_lambda_s0_scipy():
    rng = np.random.default_rng(1)
    for theta in list(rng.uniform(0.01, math.pi - 0.01, 5)) + [1e-4, 3.14]:
        for m in (0, 1, 5, 17, 40):
            lam = oracle.lam(60, m, 0, theta)
            for l in range(m, 61):
                ref = sph_harm_y(l, m, theta, 0.0).real
                assert abs(lam[l] - ref) <= 1e-13 * max(1.0, abs(ref)), (theta, l, m)


def _mp_lambda_s0(lmax, m, theta, dps=50):
    """Normalised scalar recurrence in 50-digit arithmetic (unbounded exponent).
    Start: lambda_mm = (-1)^m sqrt((2m+1)/(4pi) prod_{k=1}^m (2k-1)/(2k)) sin^m."""
    with mpmath.workdps(dps):
        th = mpmath.mpf(theta)
        x, s = mpmath.cos(th), mpmath.sin(th)
        prod = mpmath.mpf(1)
        for k in range(1, m + 1):
            prod *= mpmath.mpf(2 * k - 1) / (2 * k)
        lm = (-1) ** m * mpmath.sqrt((2 * m + 1) / (4 * mpmath.pi) * prod) * s ** m
        out = {m: lm}
        prev, cur = mpmath.mpf(0), lm
        for l in range(m, lmax):
            l1 = l + 1
            a1 = mpmath.sqrt(mpmath.mpf(4 * l1 * l1 - 1) / (l1 * l1 - m * m))
            b0 = mpmath.sqrt(mpmath.mpf(l * l - m * m) / (4 * l * l - 1)) if l > m else 0
            nxt = a1 * (x * cur - b0 * prev)
            prev, cur = cur, nxt
            out[l1] = cur
        return out


@pytest.mark.parametrize("lmax,m,theta", [
    (4095, 0, 0.05), (4095, 3000, 0.9), (4095, 2000, 0.6), (4095, 4095, math.pi / 2),
    (4095, 700, 0.2), (2047, 1500, 2.5), (4095, 100, 5.9e-4), (4095, 4000, 1.3),
])
def test_lambda_s0_high_precision(lmax, m, theta):
    """The long recursion (l up to 4095, values down to 1e-13000) against a
    50-digit recursion of a different (normalised Legendre) form."""
    lam = oracle.lam(lmax, m, 0, theta)
    ref = _mp_lambda_s0(lmax, m, theta)
    ls = sorted(ref)
    refv = np.array([float(ref[l]) for l in ls])
    got = lam[ls]
    scale = np.max(np.abs(refv))
    assert scale > 0
    err = np.max(np.abs(got - refv)) / scale
    assert err < 1e-13, err


def _mp_lambda_spin2(lmax, m, theta, dps=50):
    """+-2 lambda from the scalar harmonics in 50-digit arithmetic, by applying
    the spin-raising operator twice to Y_lm (a route that shares nothing with
    Eq. 11): with Y = lambda_l (scalar, from _mp_lambda_s0), x = cos, s = sin,
      s dY/dtheta = l x Y - sqrt((2l+1)/(2l-1)) sqrt(l^2 - m^2) lambda_{l-1},
      base  = -l(l+1) Y - 2 (x/s) dY/dtheta + 2 m^2/s^2 Y,
      cross = (2m/s) (dY/dtheta - (x/s) Y),
      +-2 lambda = (base -+ cross) / sqrt((l-1) l (l+1) (l+2)).
    Returns {l: (lambda_{+2}, lambda_{-2})}."""
    lam = _mp_lambda_s0(lmax, m, theta, dps)
    out = {}
    with mpmath.workdps(dps):
        th = mpmath.mpf(theta)
        x, s = mpmath.cos(th), mpmath.sin(th)
        for l in range(max(m, 2), lmax + 1):
            y = lam[l]
            yp = lam[l - 1] if l - 1 >= m else mpmath.mpf(0)
            dy = (l * x * y - mpmath.sqrt(mpmath.mpf(2 * l + 1) / (2 * l - 1))
                  * mpmath.sqrt(mpmath.mpf(l * l - m * m)) * yp) / s
            base = -l * (l + 1) * y - 2 * x / s * dy + 2 * m * m / (s * s) * y
            cross = 2 * m / s * (dy - x / s * y)
            norm = 1 / mpmath.sqrt(mpmath.mpf((l - 1) * l * (l + 1) * (l + 2)))
            out[l] = (norm * (base - cross), norm * (base + cross))
    return out


def test_spin2_from_scalar_matches_explicit_sum():
    """The spin-raising route of _mp_lambda_spin2 equals Wigner's explicit sum
    with Eq. 10's normalisation at low degrees (fixes its sign convention)."""
    for theta in (0.3, 1.1, 2.5):
        for m in (0, 1, 3, 7):
            ref = _mp_lambda_spin2(16, m, theta)
            for l in range(max(m, 2), 17):
                for k, s in enumerate((2, -2)):
                    d = _mp_d_explicit(l, -m, s, theta)
                    direct = (-1) ** m * math.sqrt((2 * l + 1) / FOURPI) * d
                    assert abs(float(ref[l][k]) - direct) < 1e-13, (theta, m, l, s)


@pytest.mark.parametrize("theta", [5.9e-4, 0.05, 1.3])
@pytest.mark.parametrize("m", [0, 1, 2, 3, 2000, 4095])
def test_lambda_s2_high_precision(theta, m):
    """The oracle's spin +-2 recursion (Eq. 11, extended exponent) up to
    l = 4095 against the 50-digit spin-raising route from the scalar
    harmonics; columns that lie entirely below the double range must come out
    as exact zeros.  Tolerance: 1e-13 normwise, except at the polar-most
    colatitude, where Eq. 11 sees theta only through x = cos theta, which
    holds theta to an absolute precision of about u / theta (u = 2^-64, the
    long double unit): at theta = 5.9e-4 that is 9e-17, and the phase of a
    degree-4095 column moves by l times that, 4e-13."""
    lmax = 4095
    tol = 5e-13 if theta < 0.01 else 1e-13
    ref = _mp_lambda_spin2(lmax, m, theta)
    ls = sorted(ref)
    for k, s in enumerate((2, -2)):
        lam = oracle.lam(lmax, m, s, theta)
        refv = np.array([float(ref[l][k]) for l in ls])
        got = lam[ls]
        scale = np.max(np.abs(refv))
        if scale == 0.0:
            assert np.all(got == 0.0), (s, m, theta)
            continue
        err = np.max(np.abs(got - refv)) / scale
        assert err < tol, (s, err)


def test_lambda_s0_legenp_sample():
    """mpmath's associated Legendre function at one mid-latitude sample."""
    l, m, theta = 1200, 500, 0.8
    lam = oracle.lam(l, m, 0, theta)[l]
    with mpmath.workdps(40):
        p = mpmath.legenp(l, m, mpmath.cos(mpmath.mpf(theta)))   # includes (-1)^m
        norm = mpmath.sqrt((2 * l + 1) / (4 * mpmath.pi) * mpmath.factorial(l - m)
                           / mpmath.factorial(l + m))
        ref = float(norm * p)
    assert abs(lam - ref) <= 1e-12 * abs(ref)


@pytest.mark.parametrize("theta", [1e-3, 0.4, 1.5, 2.9])
def test_addition_theorem_s0(theta):
    lmax = 300
    tot = np.zeros(lmax + 1)
    for m in range(-lmax, lmax + 1):
        tot += oracle.lam(lmax, m, 0, theta) ** 2
    ref = (2 * np.arange(lmax + 1) + 1) / FOURPI
    assert np.max(np.abs(tot - ref) / ref) < 1e-13


# ---------------------------------------------------------------- lambda, s=+-2
def _d2(k, c, s):
    """d^2_{2,k}(theta) (Wigner small-d table, l = 2), s = sin(theta)."""
    return {2: (1 + c) ** 2 / 4, 1: -(1 + c) * s / 2, 0: math.sqrt(3 / 8) * s * s,
            -1: -(1 - c) * s / 2, -2: (1 - c) ** 2 / 4}[k]


@pytest.mark.parametrize("theta", [1e-3, 0.7, 1.9, math.pi - 1e-3])
def test_lambda_s2_closed_forms(theta):
    c, s = math.cos(theta), math.sin(theta)
    n = math.sqrt(5 / FOURPI)
    for m in range(-2, 3):
        lp = oracle.lam(3, m, 2, theta)[2]
        lm = oracle.lam(3, m, -2, theta)[2]
        # Eq. 10 with the table: 2_lambda_2m = n d^2_{2,-m}, -2_lambda_2m = (-1)^m n d^2_{2,m}
        assert abs(lp - n * _d2(-m, c, s)) < 2e-15, m
        assert abs(lm - (-1) ** m * n * _d2(m, c, s)) < 2e-15, m
    assert abs(oracle.lam(2, 0, 2, theta)[2] - math.sqrt(15 / (32 * math.pi)) * s * s) < 2e-15


@pytest.mark.parametrize("theta", [0.02, 0.9, 2.2])
def test_lambda_s2_m0_from_legendre(theta):
    """+-2 lambda_l0 = sqrt((2l+1)/4pi) sqrt((l-2)!/(l+2)!) P_l^2(cos theta)."""
    lmax = 80
    x = math.cos(theta)
    for s in (2, -2):
        lam = oracle.lam(lmax, 0, s, theta)
        for l in range(2, lmax + 1):
            ref = (math.sqrt((2 * l + 1) / FOURPI)
                   * math.exp(0.5 * (math.lgamma(l - 1) - math.lgamma(l + 3)))
                   * lpmv(2, l, x))
            assert abs(lam[l] - ref) <= 1e-12 * max(1e-3, abs(ref)), (s, l)


@pytest.mark.parametrize("theta", [3e-3, 0.5, 1.4, 2.6])
def test_addition_theorem_s2(theta):
    lmax = 200
    for s in (2, -2):
        tot = np.zeros(lmax + 1)
        for m in range(-lmax, lmax + 1):
            tot += oracle.lam(lmax, m, s, theta) ** 2
        ls = np.arange(2, lmax + 1)
        ref = (2 * ls + 1) / FOURPI
        assert np.max(np.abs(tot[2:] - ref) / ref) < 1e-13


@pytest.mark.parametrize("theta", [0.1, 1.2])
def test_parity_relation(theta):
    """s_lambda_lm(pi - theta) = (-1)^(l+m) (-s)_lambda_lm(theta)."""
    lmax = 120
    for s in (0, 2, -2):
        for m in (-7, 0, 3, 50):
            a = oracle.lam(lmax, m, s, math.pi - theta)
            b = oracle.lam(lmax, m, -s, theta)
            sign = (-1.0) ** (np.arange(lmax + 1) + m)
            assert np.max(np.abs(a - sign * b)) < 1e-13


def _mp_d_explicit(j, mp, mm, beta):
    with mpmath.workdps(40):
        c, s = mpmath.cos(mpmath.mpf(beta) / 2), mpmath.sin(mpmath.mpf(beta) / 2)
        f = mpmath.factorial
        tot = mpmath.mpf(0)
        for k in range(0, 2 * j + 1):
            args = (j + mm - k, k, j - k - mp, k - mm + mp)
            if min(args) < 0:
                continue
            t = (-1) ** (k - mm + mp) * mpmath.sqrt(f(j + mp) * f(j - mp) * f(j + mm) * f(j - mm))
            t /= f(args[0]) * f(args[1]) * f(args[2]) * f(args[3])
            tot += t * c ** (2 * j - 2 * k + mm - mp) * s ** (2 * k - mm + mp)
        return float(tot)


def test_recursion_against_explicit_sum():
    """Every degree from the Eq. 11 recursion equals Wigner's full explicit sum
    (the oracle only uses the sum at the lowest degree)."""
    beta = 0.83
    for s in (0, 2, -2, 1, -1, 3, -3):
        for m in (-5, -2, 0, 1, 4):
            lam = oracle.lam(24, m, s, beta)
            for l in range(max(abs(m), abs(s)), 25):
                d = _mp_d_explicit(l, -m, s, beta)
                ref = (-1) ** m * math.sqrt((2 * l + 1) / FOURPI) * d
                assert abs(lam[l] - ref) < 1e-13, (s, m, l)


def test_recursion_against_explicit_sum_spin37():
    """The spin the paper's tests use: s = 37 at degrees up to 60."""
    beta = 1.31
    for s in (37, -37):
        for m in (0, 5, -20, 40):
            lam = oracle.lam(60, m, s, beta)
            for l in range(max(abs(m), abs(s)), 61, 7):
                d = _mp_d_explicit(l, -m, s, beta)
                ref = (-1) ** m * math.sqrt((2 * l + 1) / FOURPI) * d
                assert abs(lam[l] - ref) < 1e-13, (s, m, l)


@pytest.mark.parametrize("s", [1, 3, 37])
def test_addition_theorem_any_spin(s):
    """sum_m |s_lambda_lm|^2 = (2l+1)/(4 pi) for every l >= s."""
    lmax = 160
    for theta in (0.05, 1.0, 2.5):
        for sg in (s, -s):
            tot = np.zeros(lmax + 1)
            for m in range(-lmax, lmax + 1):
                tot += oracle.lam(lmax, m, sg, theta) ** 2
            ls = np.arange(s, lmax + 1)
            ref = (2 * ls + 1) / FOURPI
            assert np.max(np.abs(tot[s:] - ref) / ref) < 1e-13


def test_parity_relation_odd_spin():
    """s_lambda_lm(pi - theta) = (-1)^(l+m) (-s)_lambda_lm(theta) for odd s, and
    -s_lambda_lm = (-1)^(s+m) s_lambda_l,-m (the relation behind the (-1)^s of
    the real-field Q - iU)."""
    lmax, theta = 80, 0.7
    for s in (1, 3, -3):
        for m in (-6, 0, 5, 33):
            a = oracle.lam(lmax, m, s, math.pi - theta)
            b = oracle.lam(lmax, m, -s, theta)
            sign = (-1.0) ** (np.arange(lmax + 1) + m)
            assert np.max(np.abs(a - sign * b)) < 1e-13
            c = oracle.lam(lmax, -m, s, theta)
            assert np.max(np.abs(b - (-1.0) ** (s + m) * c)) < 1e-13


def test_wigner_d_orthogonality_and_limits():
    j = 9
    beta = 1.234
    D = np.array([[oracle.wigner_d(j, a, b, beta) for b in range(-j, j + 1)]
                  for a in range(-j, j + 1)])
    assert np.max(np.abs(D.T @ D - np.eye(2 * j + 1))) < 1e-13
    D0 = np.array([[oracle.wigner_d(j, a, b, 0.0) for b in range(-j, j + 1)]
                   for a in range(-j, j + 1)])
    assert np.max(np.abs(D0 - np.eye(2 * j + 1))) < 1e-15
    # d^j_{m'm}(pi) = (-1)^(j-m) delta_{m',-m}
    Dp = np.array([[oracle.wigner_d(j, a, b, math.pi) for b in range(-j, j + 1)]
                   for a in range(-j, j + 1)])
    ref = np.zeros_like(Dp)
    for ib, b in enumerate(range(-j, j + 1)):
        ref[2 * j - ib, ib] = (-1) ** (j - b)
    assert np.max(np.abs(Dp - ref)) < 1e-13


# ---------------------------------------------------------------- transforms
def _brute_s0(geom, lmax, alm):
    out = np.zeros(geom.npix)
    for y in range(geom.nrings):
        phi = geom.phi0[y] + 2 * math.pi * np.arange(geom.nphi[y]) / geom.nphi[y]
        acc = np.zeros(geom.nphi[y])
        for m in range(0, lmax + 1):
            for l in range(m, lmax + 1):
                a = alm[si.alm_index(lmax, l, m)]
                yv = sph_harm_y(l, m, geom.theta[y], phi)
                v = (a[0] + 1j * a[1]) * yv
                acc += v.real if m == 0 else 2 * v.real
        out[geom.ofs[y]:geom.ofs[y] + geom.nphi[y]] = acc
    return out


def test_synthesis_brute_force_s0():
    lmax = 7
    g = si.gauss_geometry(9, 17, phi0=0.3)
    a = si.random_alm(lmax, lmax, 1, 0, spectrum="unit", tag=5)
    mp = oracle.synthesis(g, lmax, lmax, 0, a)
    ref = _brute_s0(g, lmax, a[0, 0])
    assert np.max(np.abs(mp[0, 0] - ref)) < 1e-13


def test_synthesis_aliasing_s0():
    """Rings with fewer pixels than 2 mmax + 1 (Eq. 3 aliases, it does not truncate)."""
    lmax = 8
    g = si.healpix_geometry(2)          # rings with 4, 8 pixels; lmax 8 aliases
    a = si.random_alm(lmax, lmax, 1, 0, spectrum="unit", tag=6)
    mp = oracle.synthesis(g, lmax, lmax, 0, a)
    ref = _brute_s0(g, lmax, a[0, 0])
    assert np.max(np.abs(mp[0, 0] - ref)) < 1e-13


def test_synthesis_spin2_single_modes():
    """E_20 = 1 gives Q = -sqrt(15/32pi) sin^2, U = 0; B_20 = 1 gives Q = 0,
    U = -sqrt(15/32pi) sin^2 (HEALPix E/B convention)."""
    lmax = 4
    g = si.gauss_geometry(6, 9, phi0=0.1)
    n = si.nalm(lmax, lmax)
    k = math.sqrt(15 / (32 * math.pi))
    for comp in (0, 1):
        a = np.zeros((1, 2, n, 2))
        a[0, comp, si.alm_index(lmax, 2, 0), 0] = 1.0
        mp = oracle.synthesis(g, lmax, lmax, 2, a)
        ref = np.repeat(-k * np.sin(g.theta) ** 2, g.nphi)
        assert np.max(np.abs(mp[0, comp] - ref)) < 1e-14
        assert np.max(np.abs(mp[0, 1 - comp])) < 1e-14


def test_synthesis_spin2_brute_force():
    """Q + iU = sum_{l,m} 2_a_lm 2_lambda_lm e^{i m phi} summed pixel by pixel
    with lambda from the closed forms at l = 2 and the m = 0 Legendre relation."""
    lmax = 2
    g = si.gauss_geometry(5, 7, phi0=0.2)
    a = si.random_alm(lmax, lmax, 1, 2, spectrum="unit", tag=9)
    mp = oracle.synthesis(g, lmax, lmax, 2, a)
    n5 = math.sqrt(5 / FOURPI)
    for y in range(g.nrings):
        c, s = math.cos(g.theta[y]), math.sin(g.theta[y])
        phi = g.phi0[y] + 2 * math.pi * np.arange(g.nphi[y]) / g.nphi[y]
        acc = np.zeros(g.nphi[y], dtype=complex)
        for m in range(-2, 3):
            am = abs(m)
            E = a[0, 0, si.alm_index(lmax, 2, am)]
            B = a[0, 1, si.alm_index(lmax, 2, am)]
            E = E[0] + 1j * (E[1] if am else 0.0)
            B = B[0] + 1j * (B[1] if am else 0.0)
            if m < 0:
                E, B = (-1) ** am * np.conj(E), (-1) ** am * np.conj(B)
            acc += -(E + 1j * B) * n5 * _d2(-m, c, s) * np.exp(1j * m * phi)
        sl = slice(g.ofs[y], g.ofs[y] + g.nphi[y])
        assert np.max(np.abs(mp[0, 0, sl] - acc.real)) < 1e-14
        assert np.max(np.abs(mp[0, 1, sl] - acc.imag)) < 1e-14


def test_phases_against_numpy_fft():
    """The exported F phases and a numpy inverse real FFT reproduce the map;
    the exported G phases equal a numpy forward FFT of the map (Eqs. 3, 6)."""
    lmax = 20
    g = si.gauss_geometry(21, 45, phi0=0.37)
    a = si.random_alm(lmax, lmax, 1, 0, tag=3)
    mp, F = oracle.synthesis(g, lmax, lmax, 0, a, want_phases=True)
    _, G = oracle.analysis(g, lmax, lmax, 0, mp, want_phases=True)
    ms = np.arange(lmax + 1)
    for y in range(g.nrings):
        N = int(g.nphi[y])
        c = (F[0, 0, y, :, 0] + 1j * F[0, 0, y, :, 1]) * np.exp(1j * ms * g.phi0[y])
        spec = np.zeros(N // 2 + 1, dtype=complex)
        spec[:lmax + 1] = c
        ring = np.fft.irfft(spec, n=N) * N
        # irfft halves the weight of bins 1.. relative to the Hermitian sum: m>0 twice
        ring_ref = np.real(c[0]) + 2 * np.real(
            np.exp(2j * math.pi * np.outer(np.arange(N), ms[1:]) / N) @ c[1:])
        assert np.max(np.abs(ring - ring_ref)) < 1e-12
        sl = slice(g.ofs[y], g.ofs[y] + N)
        assert np.max(np.abs(mp[0, 0, sl] - ring_ref)) < 1e-12
        fw = np.fft.fft(mp[0, 0, sl])[:lmax + 1] * g.weight[y] * np.exp(-1j * ms * g.phi0[y])
        gg = G[0, 0, y, :, 0] + 1j * G[0, 0, y, :, 1]
        assert np.max(np.abs(fw - gg)) < 1e-12


@pytest.mark.parametrize("spin", [0, 1, 2, 3, 4])
def test_gauss_round_trip_small(spin):
    lmax = 31
    g = si.gauss_geometry(lmax + 1, 2 * lmax + 1, phi0=0.25)
    a = si.random_alm(lmax, lmax, 2, spin, spectrum="unit", tag=11)
    b = oracle.analysis(g, lmax, lmax, spin, oracle.synthesis(g, lmax, lmax, spin, a))
    assert np.max(np.abs(a - b)) / np.max(np.abs(a)) < 1e-13


def test_gauss_round_trip_gl127():
    """The small workload: lmax 127, 128 rings x 255 px; exact quadrature."""
    lmax = 127
    g = si.gauss_geometry(128, 255)
    a = si.random_alm(lmax, lmax, 1, 0, spectrum="unit")
    b = oracle.analysis(g, lmax, lmax, 0, oracle.synthesis(g, lmax, lmax, 0, a))
    err = np.max(np.abs(a - b)) / np.max(np.abs(a))
    assert err < 1e-12, err


@pytest.mark.parametrize("spin,lmax", [(0, 63), (2, 63), (37, 63), (0, 127)])
def test_sht_pair_accuracy(spin, lmax):
    """Sect. 5, evaluation of SHT pairs: uniform [-1, 1) coefficients (Im a_l0 = 0)
    through a synthesis onto the reduced Gauss-Legendre grid and back.  The errors
    stay near the double-precision limit, the relative rms error below u (lmax + 1)
    and the largest error below u (lmax + 1)^(3/2), u = 2^-53 (the growth laws the
    paper reports, with unit constant).  One ring weight off by 1e-4, or any
    normalisation error that synthesis and analysis share, puts the rms error
    orders of magnitude above the bound."""
    g = si.reduced_gauss_geometry(lmax + 1, 2 * lmax + 2, lmax, lmax, spin)
    assert g.nphi.sum() < (lmax + 1) * (2 * lmax + 1) or lmax < 100
    a = si.random_alm(lmax, lmax, 1, spin, spectrum="uniform", tag=900 + spin)
    b = oracle.analysis(g, lmax, lmax, spin, oracle.synthesis(g, lmax, lmax, spin, a))
    d = b - a
    u = 2.0 ** -53
    rms = math.sqrt(float(np.sum(d * d)) / float(np.sum(a * a)))
    mx = float(np.max(np.hypot(d[..., 0], d[..., 1])))
    assert rms <= u * (lmax + 1), rms
    assert mx <= u * (lmax + 1) ** 1.5, mx


@pytest.mark.parametrize("spin", [0, 1, 2, 3])
def test_adjoint_dot_product(spin):
    """<Y a, g> = sum_lm fac_m Re(conj(a_lm) (Y^T g)_lm), fac_0 = 1, fac_m>0 = 2,
    on a HEALPix grid (no quadrature exactness involved)."""
    lmax = 12
    geom = si.healpix_geometry(4)
    ncomp = 2 if spin else 1
    a = si.random_alm(lmax, lmax, 1, spin, spectrum="unit", tag=21)
    gmap = si.random_map(geom, 1, ncomp, tag=22)
    ya = oracle.synthesis(geom, lmax, lmax, spin, a)
    yt = oracle.adjoint_synthesis(geom, lmax, lmax, spin, gmap)
    _, ms = si.lm_arrays(lmax, lmax)
    fac = np.where(ms == 0, 1.0, 2.0)
    lhs = float(np.sum(ya * gmap))
    rhs = float(np.sum(fac[None, None, :] * (a[..., 0] * yt[..., 0] + a[..., 1] * yt[..., 1])))
    assert abs(lhs - rhs) < 1e-12 * max(1.0, abs(lhs))


def test_sampled_modes_match_full():
    """Ring subsets (synthesis) and m subsets (analysis) equal the full run."""
    lmax = 24
    g = si.healpix_geometry(8)
    a = si.random_alm(lmax, lmax, 2, 0, tag=31)
    full = oracle.synthesis(g, lmax, lmax, 0, a)
    rings = [0, 5, 16, 30]
    part = oracle.synthesis(g, lmax, lmax, 0, a, rings=rings)
    for y in rings:
        sl = slice(g.ofs[y], g.ofs[y] + g.nphi[y])
        assert np.array_equal(part[:, :, sl], full[:, :, sl])
    A = oracle.analysis(g, lmax, lmax, 0, full)
    ms = [0, 3, 24]
    B = oracle.analysis(g, lmax, lmax, 0, full, ms=ms)
    ls, mm = si.lm_arrays(lmax, lmax)
    sel = np.isin(mm, ms)
    assert np.array_equal(A[:, :, sel], B[:, :, sel])
    assert np.all(B[:, :, ~sel] == 0)


def test_ignored_inputs():
    """Im(a_l0) and (spin 2) l < 2 coefficients do not influence the map."""
    lmax = 6
    g = si.gauss_geometry(8, 13)
    for spin in (0, 2):
        a = si.random_alm(lmax, lmax, 1, spin, spectrum="unit", tag=41)
        b = a.copy()
        ls, ms = si.lm_arrays(lmax, lmax)
        b[:, :, ms == 0, 1] = 7.0
        if spin:
            b[:, :, ls < 2, :] = 3.0
        assert np.array_equal(oracle.synthesis(g, lmax, lmax, spin, a),
                              oracle.synthesis(g, lmax, lmax, spin, b))


# ---------------------------------------------------------------- first derivatives (Sect. 4.3)

def _rings_geometry(theta, nphi, phi0):
    theta = np.asarray(theta, dtype=np.float64)
    n = len(theta)
    nphi = np.full(n, nphi, dtype=np.int64)
    phi0 = np.broadcast_to(np.asarray(phi0, dtype=np.float64), (n,)).copy()
    ofs = np.arange(n, dtype=np.int64) * nphi[0]
    return si.Geometry(theta, nphi, phi0, np.ones(n), ofs, 1)


def test_deriv_closed_forms():
    """df/dtheta and df/(sin theta dphi) of single low-degree modes, written
    out from Y_10, Y_11, Y_20, Y_21 (Condon-Shortley), including both poles
    (where df/(sin theta dphi) takes its limit)."""
    theta = np.array([0.0, 0.2, 1.0, 0.5 * math.pi, 2.3, math.pi])
    nphi = 7
    g = _rings_geometry(theta, nphi, 0.3)
    th = np.repeat(theta, nphi)
    ph = np.concatenate([0.3 + 2 * math.pi * np.arange(nphi) / nphi] * len(theta))
    lmax = 3
    n = si.nalm(lmax, lmax)
    c10, c11 = math.sqrt(3 / (4 * math.pi)), math.sqrt(3 / (8 * math.pi))
    c20, c21 = math.sqrt(5 / (16 * math.pi)), math.sqrt(15 / (8 * math.pi))
    cases = [  # (l, m, re, im) -> (df/dtheta, df/(sin theta dphi))
        (1, 0, 1.0, 0.0, -c10 * np.sin(th), 0 * th),
        (1, 1, 1.0, 0.0, -2 * c11 * np.cos(th) * np.cos(ph), 2 * c11 * np.sin(ph)),
        (1, 1, 0.0, 1.0, 2 * c11 * np.cos(th) * np.sin(ph), 2 * c11 * np.cos(ph)),
        (2, 0, 1.0, 0.0, -6 * c20 * np.cos(th) * np.sin(th), 0 * th),
        (2, 1, 1.0, 0.0, -2 * c21 * np.cos(2 * th) * np.cos(ph), 2 * c21 * np.cos(th) * np.sin(ph)),
    ]
    for l, m, re, im, dth, dph in cases:
        a = np.zeros((1, 1, n, 2))
        a[0, 0, si.alm_index(lmax, l, m)] = (re, im)
        d = oracle.deriv_synthesis(g, lmax, lmax, a)
        assert np.max(np.abs(d[0, 0] - dth)) < 1e-14, (l, m, re, im)
        assert np.max(np.abs(d[0, 1] - dph)) < 1e-14, (l, m, re, im)


def test_deriv_finite_differences():
    """Against fourth-order central differences of the spin-0 synthesis in
    theta and phi (random coefficients up to l = 20, rings in both
    hemispheres and close to a pole)."""
    lmax, h = 20, 2e-4
    theta = np.array([0.03, 0.4, 1.2, 1.9, 2.7, 3.1])
    nphi, phi0 = 45, 0.17
    a = si.random_alm(lmax, lmax, 2, 0, spectrum="unit", tag=61)
    d = oracle.deriv_synthesis(_rings_geometry(theta, nphi, phi0), lmax, lmax, a)

    def f(dt, dp):
        return oracle.synthesis(_rings_geometry(theta + dt, nphi, phi0 + dp), lmax, lmax, 0, a)[:, 0]

    def d4(step):
        return (-step(2 * h) + 8 * step(h) - 8 * step(-h) + step(-2 * h)) / (12 * h)

    dth = d4(lambda x: f(x, 0.0))
    dph = d4(lambda x: f(0.0, x)) / np.repeat(np.sin(theta), nphi)[None]
    scale = np.max(np.abs(d))
    assert np.max(np.abs(d[:, 0] - dth)) < 1e-8 * scale
    assert np.max(np.abs(d[:, 1] - dph)) < 1e-8 * scale


def test_deriv_adjoint_dot_product():
    """<D a, g> = sum_lm fac_m Re(conj(a_lm) (D^T g)_lm) for the derivative
    synthesis D and deriv_adjoint, on a HEALPix grid."""
    lmax = 12
    geom = si.healpix_geometry(4)
    a = si.random_alm(lmax, lmax, 1, 0, spectrum="unit", tag=62)
    gmap = si.random_map(geom, 1, 2, tag=63)
    lhs = float(np.sum(oracle.deriv_synthesis(geom, lmax, lmax, a) * gmap))
    dt = oracle.deriv_adjoint(geom, lmax, lmax, gmap)
    _, ms = si.lm_arrays(lmax, lmax)
    fac = np.where(ms == 0, 1.0, 2.0)
    rhs = float(np.sum(fac[None, None, :] * (a[..., 0] * dt[..., 0] + a[..., 1] * dt[..., 1])))
    assert abs(lhs - rhs) < 1e-12 * max(1.0, abs(lhs))


# ---------------------------------------------------------------- real harmonics (Sect. 4.5)

def test_real_harmonics_closed_forms():
    """R_11 = sqrt(2) Re Y_11 = -sqrt(3/4pi) sin(theta) cos(phi),
    R_1,-1 = sqrt(2) Im Y_11 = -sqrt(3/4pi) sin(theta) sin(phi), R_10 = Y_10."""
    theta = np.array([0.3, 1.2, 2.5])
    nphi = 9
    g = _rings_geometry(theta, nphi, 0.4)
    th = np.repeat(theta, nphi)
    ph = np.concatenate([0.4 + 2 * math.pi * np.arange(nphi) / nphi] * len(theta))
    lmax = 2
    c = math.sqrt(3 / (4 * math.pi))
    for (l, m, slot), ref in [((1, 1, 0), -c * np.sin(th) * np.cos(ph)),
                              ((1, 1, 1), -c * np.sin(th) * np.sin(ph)),
                              ((1, 0, 0), c * np.cos(th))]:
        r = np.zeros((1, 1, si.nalm(lmax, lmax), 2))
        r[0, 0, si.alm_index(lmax, l, m), slot] = 1.0
        f = oracle.synthesis_real(g, lmax, lmax, 0, r)[0, 0]
        assert np.max(np.abs(f - ref)) < 1e-14, (l, m, slot)


@pytest.mark.parametrize("spin", [0, 2])
def test_real_harmonics_orthonormal_and_plain_adjoint(spin):
    """Under exact Gauss-Legendre quadrature the real harmonics are orthonormal
    (analysis_real inverts synthesis_real), and adjoint_synthesis_real is the
    plain transpose: <Y r, x> = <r, Y^T x> with no m-dependent factors."""
    lmax = 10
    g = si.gauss_geometry(lmax + 1, 2 * lmax + 1, 0.2)
    r = si.random_alm(lmax, lmax, 1, spin, spectrum="unit", tag=71)
    ls, ms = si.lm_arrays(lmax, lmax)
    r[:, :, ms == 0, 1] = 0.0       # no slot for r_l,-0
    if spin:
        r[:, :, ls < spin, :] = 0.0
    back = oracle.analysis_real(g, lmax, lmax, spin, oracle.synthesis_real(g, lmax, lmax, spin, r))
    assert np.max(np.abs(back - r)) < 1e-13
    h = si.healpix_geometry(4)
    x = si.random_map(h, 1, 2 if spin else 1, tag=72)
    lhs = float(np.sum(oracle.synthesis_real(h, lmax, lmax, spin, r) * x))
    rhs = float(np.sum(r * oracle.adjoint_synthesis_real(h, lmax, lmax, spin, x)))
    assert abs(lhs - rhs) < 1e-12 * max(1.0, abs(lhs))
