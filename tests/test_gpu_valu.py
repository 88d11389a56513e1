"""The vector-unit Legendre kernels (spin 0 with one or two transforms and
spin > 0 with one: the default there) against the oracle and against the
matrix-core kernels of the same plan (set through the tuning), including the
gradient mode, the derivative maps, batches and ragged sizes."""
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
    # name: (geometry, lmax, mmax, ntrans)
    "gl_j1": (lambda: si.gauss_geometry(48, 95, 0.2), 47, 47, 1),
    "gl_j2_mmax": (lambda: si.gauss_geometry(40, 81), 39, 25, 2),
    "hp_j1_alias": (lambda: si.healpix_geometry(16), 47, 47, 1),
    "hp_j3_ragged": (lambda: si.healpix_geometry(8), 23, 23, 3),   # groups of two, the last one ragged
    "gl_lmax0": (lambda: si.gauss_geometry(1, 1), 0, 0, 1),
    "gl_j1_long": (lambda: si.gauss_geometry(200, 399), 199, 199, 1),
    # many rings at a small lmax: two slots per lane in the synthesis, four in
    # the analysis (two with fewer than eight 64-slot units), tiles of several
    # passes of the analysis work group, most polar tiles skipped at the higher m
    "gl_j1_k4": (lambda: si.gauss_geometry(1000, 129, 0.1), 60, 60, 1),
    "gl_j2_k4": (lambda: si.gauss_geometry(1000, 129), 60, 45, 2),
    "gl_j2_k2": (lambda: si.gauss_geometry(300, 129), 60, 60, 2),   # 150 slots: three 64-slot units
    "gl_j1_k4_passes": (lambda: si.gauss_geometry(2100, 67), 33, 33, 1),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_valu_against_oracle_and_matrix_path(name):
    sht = _sht()
    build, lmax, mmax, ntrans = CASES[name]
    g = build()
    p = sht.Plan(sht.Geometry.from_inputs(g), lmax, mmax, spin=0, ntrans=ntrans)
    if ntrans <= 2:
        assert p.tuning()["valu"] == 1, "the vector path is the default for one or two transforms"
    p.set_tuning(valu=1)
    a = si.random_alm(lmax, mmax, ntrans, 0, tag=17)
    d_a = to_dev(a)
    mp = to_host(p.alm2map(d_a))
    ref_map = oracle.synthesis(g, lmax, mmax, 0, a)
    assert rel_err(mp, ref_map) < TOL64
    back = to_host(p.map2alm(to_dev(ref_map)))
    ref_alm = oracle.analysis(g, lmax, mmax, 0, ref_map)
    assert rel_err(back, ref_alm) < TOL64
    grad = to_host(p.alm2map_grad(to_dev(ref_map)))
    ref_g = oracle.adjoint_synthesis(g, lmax, mmax, 0, ref_map)
    ref_g = ref_g * np.where(si.lm_arrays(lmax, mmax)[1] == 0, 1.0, 2.0)[None, None, :, None]
    assert rel_err(grad, ref_g) < TOL64
    # the matrix-core kernels give the same sums up to rounding order
    p.set_tuning(valu=0)
    assert rel_err(to_host(p.alm2map(d_a)), mp) < 1e-13
    assert rel_err(to_host(p.map2alm(to_dev(ref_map))), back) < 1e-13


def test_valu_batch_equals_plans():
    sht = _sht()
    plans, alms = [], []
    for k, lmax in enumerate([31, 63]):
        g = si.gauss_geometry(lmax + 1, 2 * lmax + 1)
        plans.append(sht.Plan(sht.Geometry.from_inputs(g), lmax, spin=0, ntrans=1 + k))
        alms.append(to_dev(si.random_alm(lmax, lmax, 1 + k, 0, tag=30 + k)))
    b = sht.Batch(plans)
    maps = b.alm2map(alms)
    back = b.map2alm(maps)
    for p, a, mp, ab in zip(plans, alms, maps, back):
        assert np.array_equal(to_host(mp), to_host(p.alm2map(a)))
        assert np.array_equal(to_host(ab), to_host(p.map2alm(mp)))


SPIN_CASES = {
    # name: (geometry, lmax, mmax, spin, ntrans)
    "s2_gl": (lambda: si.gauss_geometry(48, 95, 0.2), 47, 47, 2, 1),
    "s1_hp_j2": (lambda: si.healpix_geometry(16), 40, 40, 1, 2),
    "s3_mmax": (lambda: si.gauss_geometry(30, 61, 0.1), 29, 20, 3, 1),   # l0 = s > m at m < 3
    "s37_gl": (lambda: si.gauss_geometry(64, 129, 0.3), 63, 63, 37, 1),
    "s2_unpaired_j3": (lambda: si.ecp_geometry(17, 41, si.ECP_FEJER1, 0.4), 20, 18, 2, 3),
    # many rings at a small lmax: two 64-slot units per lane, several passes of
    # the analysis work group, a ragged last unit (1000 rings: 500 pairs)
    "s2_k2_passes": (lambda: si.gauss_geometry(1000, 129, 0.1), 60, 60, 2, 1),
    "s1_lmax_eq_s": (lambda: si.gauss_geometry(4, 9), 1, 1, 1, 1),
}


@pytest.mark.parametrize("name", sorted(SPIN_CASES))
def test_valu_spin_against_oracle_and_matrix_path(name):
    sht = _sht()
    build, lmax, mmax, spin, ntrans = SPIN_CASES[name]
    g = build()
    p = sht.Plan(sht.Geometry.from_inputs(g), lmax, mmax, spin=spin, ntrans=ntrans)
    assert p.tuning()["valu"] == (1 if ntrans == 1 else 0), "the vector path is the default for one transform"
    p.set_tuning(valu=1)
    a = si.random_alm(lmax, mmax, ntrans, spin, tag=19 + spin)
    d_a = to_dev(a)
    mp = to_host(p.alm2map(d_a))
    ref_map = oracle.synthesis(g, lmax, mmax, spin, a)
    assert rel_err(mp, ref_map) < TOL64
    back = to_host(p.map2alm(to_dev(ref_map)))
    assert rel_err(back, oracle.analysis(g, lmax, mmax, spin, ref_map)) < TOL64
    x = si.random_map(g, ntrans, 2, tag=23)
    ref_t = oracle.adjoint_synthesis(g, lmax, mmax, spin, x)
    assert rel_err(to_host(p.adjoint(to_dev(x))), ref_t) < TOL64
    fac = np.where(si.lm_arrays(lmax, mmax)[1] == 0, 1.0, 2.0)[None, None, :, None]
    assert rel_err(to_host(p.alm2map_grad(to_dev(x))), fac * ref_t) < TOL64
    # the matrix-core kernels give the same sums up to rounding order
    p.set_tuning(valu=0)
    assert rel_err(to_host(p.alm2map(d_a)), mp) < 1e-13
    assert rel_err(to_host(p.map2alm(to_dev(ref_map))), back) < 1e-13


@pytest.mark.parametrize("geom,lmax,mmax,ntrans", [
    (lambda: si.gauss_geometry(40, 81), 39, 25, 1),
    (lambda: si.healpix_geometry(16), 40, 40, 2),
    (lambda: si.ecp_geometry(33, 64, si.ECP_CC, 0.3), 30, 30, 1),
], ids=["gl_mmax", "hp_j2", "cc_poles"])
def test_valu_derivative_maps(geom, lmax, mmax, ntrans):
    """Derivative maps on the vector kernels (E = sqrt(l (l + 1)) a, B = 0) and
    their adjoint, against the oracle and the matrix-core kernels."""
    sht = _sht()
    g = geom()
    p = sht.Plan(sht.Geometry.from_inputs(g), lmax, mmax, spin=1, ntrans=ntrans)
    p.set_tuning(valu=1)
    a = si.random_alm(lmax, mmax, ntrans, 0, tag=29)
    d = to_host(p.alm2map_deriv1(to_dev(a)))
    assert rel_err(d, oracle.deriv_synthesis(g, lmax, mmax, a)) < TOL64
    x = si.random_map(g, ntrans, 2, tag=31)
    ref = oracle.deriv_adjoint(g, lmax, mmax, x)
    adj = to_host(p.deriv1_adjoint(to_dev(x)))
    assert rel_err(adj, ref) < TOL64
    fac = np.where(si.lm_arrays(lmax, mmax)[1] == 0, 1.0, 2.0)[None, None, :, None]
    assert rel_err(to_host(p.alm2map_deriv1_grad(to_dev(x))), fac * ref) < TOL64
    p.set_tuning(valu=0)
    assert rel_err(to_host(p.alm2map_deriv1(to_dev(a))), d) < 1e-13
    assert rel_err(to_host(p.deriv1_adjoint(to_dev(x))), adj) < 1e-13


def test_valu_spin_batch_equals_plans():
    """Batches of single spin-2 transforms (vector path; each plan runs its own
    analysis launch) give the plans' results bit for bit, eager and replayed."""
    import torch
    sht = _sht()
    plans, alms = [], []
    for k, lmax in enumerate([23, 47]):
        g = si.gauss_geometry(lmax + 1, 2 * lmax + 1, 0.1 * k)
        p = sht.Plan(sht.Geometry.from_inputs(g), lmax, spin=2, ntrans=1)
        assert p.tuning()["valu"] == 1
        plans.append(p)
        alms.append(to_dev(si.random_alm(lmax, lmax, 1, 2, tag=40 + k)))
    b = sht.Batch(plans)
    s = torch.cuda.Stream()
    for stream in (None, s, s):
        with torch.cuda.stream(s if stream is not None else torch.cuda.current_stream()):
            maps = b.alm2map(alms, stream=stream)
            back = b.map2alm(maps, stream=stream)
        torch.cuda.synchronize()
        for p, a, mp, ab in zip(plans, alms, maps, back):
            assert np.array_equal(to_host(mp), to_host(p.alm2map(a)))
            assert np.array_equal(to_host(ab), to_host(p.map2alm(mp)))


@pytest.mark.parametrize("spin", [0, 2])
def test_valu_deterministic(spin):
    """Repeated runs of the vector kernels give the same bits (fixed-order
    butterfly and work-group sums, no atomics)."""
    sht = _sht()
    g = si.healpix_geometry(32)
    lmax = 80
    p = sht.Plan(sht.Geometry.from_inputs(g), lmax, spin=spin, ntrans=1)
    assert p.tuning()["valu"] == 1
    a = to_dev(si.random_alm(lmax, lmax, 1, spin, tag=61))
    m1, m2 = to_host(p.alm2map(a)), to_host(p.alm2map(a))
    assert np.array_equal(m1, m2)
    x = to_dev(m1)
    assert np.array_equal(to_host(p.map2alm(x)), to_host(p.map2alm(x)))


def test_valu_unsupported_combinations_rejected():
    sht = _sht()
    g = sht.Geometry.from_inputs(si.gauss_geometry(16, 31))
    for kw in (dict(spin=0, precision="fp32_mfma"), dict(spin=2, precision="fp32_mfma")):
        p = sht.Plan(g, 15, ntrans=1, **kw)
        assert p.tuning()["valu"] == 0
        with pytest.raises(sht.ShtError) as e:
            p.set_tuning(valu=1)
        assert e.value.status == sht.SHT_EUNSUPPORTED
