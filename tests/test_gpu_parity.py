"""GPU parity of the full transforms and of each stage against the CPU oracle.

Tolerance for the FP64 path: normwise max relative error <= 1e-11
(max|x - ref| / max|ref|), the accuracy of the FP64 recursion at l ~ 4000
(lambda_mm inherits a relative error ~ m * eps from the rounding of sin theta).
"""
import math
import zlib

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
    # name: (geometry builder, lmax, mmax, spin, ntrans)
    "gl_s0": (lambda: si.gauss_geometry(32, 63, 0.0), 31, 31, 0, 1),
    "gl_s0_j3_phi": (lambda: si.gauss_geometry(33, 67, 0.3), 31, 31, 0, 3),
    "gl_s0_mmax": (lambda: si.gauss_geometry(20, 41), 19, 11, 0, 2),
    "gl_s2": (lambda: si.gauss_geometry(24, 47, 0.1), 23, 23, 2, 2),
    "gl_s2_j5_mmax": (lambda: si.gauss_geometry(22, 45), 21, 15, 2, 5),
    "hp_s0_alias": (lambda: si.healpix_geometry(8), 23, 23, 0, 1),
    "hp_s2_alias": (lambda: si.healpix_geometry(8), 20, 20, 2, 2),
    "hp_s0_j9": (lambda: si.healpix_geometry(16), 47, 47, 0, 9),
    "gl_odd_nphi_prime": (lambda: si.gauss_geometry(40, 79), 39, 39, 0, 2),
    "gl_s2_j16": (lambda: si.gauss_geometry(16, 31), 15, 15, 2, 16),
    # ring lengths of every FFT kind: 8191 prime with 8190 = 2 3^2 5 7 13
    # (paired, no aliasing: Rader with the convolution split into two halves
    # of 4095), 7351 (prime, split Rader with 3675 = 3 5^2 7^2), 4051 (prime,
    # split Rader with 2025 = 3^4 5^2), 16382 (half length 8191, Rader), 8190
    # (half 4095 = 3^2 5 7 13, direct), 1287 = 3^2 11 13 (paired, direct odd
    # radices), 2006 (half 1003 = 17 59, Bluestein in LDS), 4097 = 17 241
    # (paired, Bluestein split in two halves), 257 (prime, Rader with a
    # power-of-two inner length), 4096 (half 2048, radix 8/4/2)
    "fft_lengths_s2": (lambda: si.mixed_geometry([8191, 16382, 8190, 1287, 2006, 7351], 0.2),
                       60, 60, 2, 2),
    "fft_lengths_s0": (lambda: si.mixed_geometry([4097, 1287, 257, 2006, 4096, 8191, 4051], 0.37),
                       45, 40, 0, 3),
    # 8191 and 4051 with mmax above half the ring length (aliased terms): the
    # unsplit Rader form over the whole length
    # (no polar skipping: the staged phases of the terms it drops would be zero)
    "fft_rader_alias": (lambda: si.mixed_geometry([8191, 4051], 0.1), 4200, 4200, 0, 1, {"polar": False}),
}


def _setup(name, precision="fp64"):
    sht = _sht()
    build, lmax, mmax, spin, ntrans = CASES[name][:5]
    kw = CASES[name][5] if len(CASES[name]) > 5 else {}
    g = build()
    geom = sht.Geometry.from_inputs(g)
    plan = sht.Plan(geom, lmax, mmax, spin=spin, ntrans=ntrans, precision=precision, **kw)
    a = si.random_alm(lmax, mmax, ntrans, spin, tag=zlib.crc32(name.encode()) % 1000)
    return g, plan, a


@pytest.mark.parametrize("name", sorted(CASES))
def test_synthesis_and_stage_F(name):
    g, plan, a = _setup(name)
    lmax, mmax, spin = plan.lmax, plan.mmax, plan.spin
    ref_map, ref_F = oracle.synthesis(g, lmax, mmax, spin, a, want_phases=True)
    F = to_host(plan.legendre_synth(to_dev(a)))
    assert rel_err(F, ref_F) < TOL64, "F phases"
    mp = to_host(plan.ring_synth(to_dev(ref_F)))
    assert rel_err(mp, ref_map) < TOL64, "ring synthesis from oracle F"
    full = to_host(plan.alm2map(to_dev(a)))
    assert rel_err(full, ref_map) < TOL64, "alm2map"


@pytest.mark.parametrize("name", sorted(CASES))
def test_analysis_and_stage_G(name):
    g, plan, a = _setup(name)
    lmax, mmax, spin = plan.lmax, plan.mmax, plan.spin
    maps = si.random_map(g, plan.ntrans, plan.ncomp, tag=3)
    ref_alm, ref_G = oracle.analysis(g, lmax, mmax, spin, maps, want_phases=True)
    G = to_host(plan.ring_anal(to_dev(maps)))
    assert rel_err(G, ref_G) < TOL64, "G phases"
    alm_from_G = to_host(plan.legendre_anal(to_dev(ref_G)))
    assert rel_err(alm_from_G, ref_alm) < TOL64, "Legendre analysis from oracle G"
    full = to_host(plan.map2alm(to_dev(maps)))
    assert rel_err(full, ref_alm) < TOL64, "map2alm"
    adj = to_host(plan.adjoint(to_dev(maps)))
    ref_adj = oracle.adjoint_synthesis(g, lmax, mmax, spin, maps)
    assert rel_err(adj, ref_adj) < TOL64, "adjoint synthesis"


def test_gl127_workload_round_trip():
    """GL 128 rings x 255 px, lmax 127, Re/Im ~ N(0,1): parity and the exact
    Gauss-Legendre round trip."""
    sht = _sht()
    g = si.gauss_geometry(128, 255)
    a = si.random_alm(127, 127, 1, 0, spectrum="unit")
    plan = sht.Plan(sht.Geometry.from_inputs(g), 127)
    mp = plan.alm2map(to_dev(a))
    back = to_host(plan.map2alm(mp))
    mp = to_host(mp)
    ref = oracle.synthesis(g, 127, 127, 0, a)
    assert rel_err(mp, ref) < TOL64
    assert rel_err(back, oracle.analysis(g, 127, 127, 0, ref)) < TOL64
    assert rel_err(back, a) < 1e-12


@pytest.mark.parametrize("name", ["gl_s2", "hp_s0_j9", "gl_s2_j16"])
def test_fp32_mfma_precision_bound(name):
    """Precision form: FP64 recursion, FP32 matrix-core products, FP64 carry.
    Stated bound: normwise max relative error <= 1e-6 against the oracle."""
    g, plan, a = _setup(name, precision="fp32_mfma")
    ref_map = oracle.synthesis(g, plan.lmax, plan.mmax, plan.spin, a)
    mp = to_host(plan.alm2map(to_dev(a)))
    assert rel_err(mp, ref_map) < 1e-6
    ref_alm = oracle.analysis(g, plan.lmax, plan.mmax, plan.spin, ref_map)
    back = to_host(plan.map2alm(to_dev(ref_map)))
    assert rel_err(back, ref_alm) < 1e-6


def test_determinism_fp64():
    g, plan, a = _setup("hp_s0_j9")
    x = to_dev(a)
    m1 = to_host(plan.alm2map(x))
    m2 = to_host(plan.alm2map(x))
    assert np.array_equal(m1, m2)
    b1 = to_host(plan.map2alm(to_dev(m1)))
    b2 = to_host(plan.map2alm(to_dev(m1)))
    assert np.array_equal(b1, b2)
