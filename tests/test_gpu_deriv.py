"""Maps of first derivatives (Sect. 4.3): df/dtheta and df/(sin theta dphi)
from spin-0 a_lm, computed by the spin-1 kernels with E = sqrt(l (l + 1)) a,
B = 0; the adjoint and the autograd backward; batches; the staged Legendre
and FFT steps; the direction's validation."""
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
    "gl": (lambda: si.gauss_geometry(64, 127, 0.2), 63, 63, 3),
    "gl_mmax": (lambda: si.gauss_geometry(40, 81), 39, 25, 1),
    "hp": (lambda: si.healpix_geometry(16), 40, 40, 2),
    "cc_poles": (lambda: si.ecp_geometry(33, 64, si.ECP_CC, 0.3), 30, 30, 2),
    "fejer1_unpaired": (lambda: si.ecp_geometry(21, 45, si.ECP_FEJER1, 0.1), 20, 20, 1),
}


def _setup(name, precision="fp64"):
    sht = _sht()
    build, lmax, mmax, ntrans = CASES[name]
    g = build()
    plan = sht.Plan(sht.Geometry.from_inputs(g), lmax, mmax, spin=1, ntrans=ntrans, precision=precision)
    a = si.random_alm(lmax, mmax, ntrans, 0, tag=600 + lmax)
    return g, plan, a


@pytest.mark.parametrize("name", sorted(CASES))
def test_deriv_synthesis_parity(name):
    g, plan, a = _setup(name)
    _, lmax, mmax, _ = CASES[name]
    d = to_host(plan.alm2map_deriv1(to_dev(a)))
    assert d.shape == plan.map_shape
    assert rel_err(d, oracle.deriv_synthesis(g, lmax, mmax, a)) < TOL64


@pytest.mark.parametrize("name", ["gl", "hp", "cc_poles"])
def test_deriv_adjoint_and_grad_parity(name):
    g, plan, a = _setup(name)
    _, lmax, mmax, ntrans = CASES[name]
    x = si.random_map(g, ntrans, 2, tag=610)
    ref = oracle.deriv_adjoint(g, lmax, mmax, x)
    adj = to_host(plan.deriv1_adjoint(to_dev(x)))
    assert adj.shape == plan.deriv_alm_shape
    assert rel_err(adj, ref) < TOL64
    _, ms = si.lm_arrays(lmax, mmax)
    fac = np.where(ms == 0, 1.0, 2.0)[None, None, :, None]
    grad = to_host(plan.alm2map_deriv1_grad(to_dev(x)))
    assert rel_err(grad, fac * ref) < TOL64


def test_deriv_adjoint_identity():
    """<D a, x> = sum over l, m >= 0 of fac_m Re(a_lm conj((D^T x)_lm)) on the GPU results."""
    g, plan, a = _setup("hp")
    _, lmax, mmax, ntrans = CASES["hp"]
    x = si.random_map(g, ntrans, 2, tag=611)
    da = to_host(plan.alm2map_deriv1(to_dev(a)))
    dt = to_host(plan.deriv1_adjoint(to_dev(x)))
    _, ms = si.lm_arrays(lmax, mmax)
    fac = np.where(ms == 0, 1.0, 2.0)
    lhs = float(np.sum(da * x))
    rhs = float(np.sum(fac[None, None, :] * (a[..., 0] * dt[..., 0] + a[..., 1] * dt[..., 1])))
    assert abs(lhs - rhs) <= 1e-12 * np.sqrt(np.sum(da * da) * np.sum(x * x))


def test_deriv_fp32_mfma_form():
    g, plan, a = _setup("gl", precision="fp32_mfma")
    d = to_host(plan.alm2map_deriv1(to_dev(a)))
    assert rel_err(d, oracle.deriv_synthesis(g, 63, 63, a)) < 1e-6
    x = si.random_map(g, 3, 2, tag=612)
    adj = to_host(plan.deriv1_adjoint(to_dev(x)))
    assert rel_err(adj, oracle.deriv_adjoint(g, 63, 63, x)) < 1e-6


def test_deriv_autograd():
    import torch
    from paper_1303_4945_amd.autograd import alm2map_deriv1
    g, plan, a = _setup("gl")
    w = si.random_map(g, 3, 2, tag=613)
    ta = to_dev(a).requires_grad_(True)
    loss = (alm2map_deriv1(ta, plan) * to_dev(w)).sum()
    loss.backward()
    _, ms = si.lm_arrays(63, 63)
    fac = np.where(ms == 0, 1.0, 2.0)[None, None, :, None]
    ref = fac * oracle.deriv_adjoint(g, 63, 63, w)
    assert rel_err(to_host(ta.grad), ref) < TOL64
    torch.cuda.synchronize()


def test_deriv_staged_steps_equal_full():
    """sht_legendre then sht_ring_fft in the derivative direction equals sht_execute."""
    sht = _sht()
    g, plan, a = _setup("gl")
    da = to_dev(a)
    full = to_host(plan.alm2map_deriv1(da))
    ph = plan._run(sht._lib.sht_legendre, sht.ALM2MAP_DERIV1, da, plan.phase_shape)
    staged = to_host(plan._run(sht._lib.sht_ring_fft, sht.ALM2MAP_DERIV1, ph, plan.map_shape))
    assert np.array_equal(staged, full)


def test_deriv_batch_equals_plans():
    sht = _sht()
    plans, alms = [], []
    for k, lmax in enumerate([15, 40]):
        g = si.gauss_geometry(lmax + 1, 2 * lmax + 1, 0.1 * k)
        plans.append(sht.Plan(sht.Geometry.from_inputs(g), lmax, spin=1, ntrans=2))
        alms.append(to_dev(si.random_alm(lmax, lmax, 2, 0, tag=620 + k)))
    b = sht.Batch(plans)
    maps = b.execute(sht.ALM2MAP_DERIV1, alms)
    for p, a, mp in zip(plans, alms, maps):
        assert np.array_equal(to_host(mp), to_host(p.alm2map_deriv1(a)))
    grads = b.execute(sht.ALM2MAP_DERIV1_GRAD, maps)
    for p, mp, gr in zip(plans, maps, grads):
        assert gr.shape == p.deriv_alm_shape
        assert np.array_equal(to_host(gr), to_host(p.alm2map_deriv1_grad(mp)))


@pytest.mark.parametrize("spin", [0, 2])
def test_deriv_needs_spin1_plan(spin):
    sht = _sht()
    g = si.gauss_geometry(8, 15)
    plan = sht.Plan(sht.Geometry.from_inputs(g), 7, spin=spin)
    a = to_dev(si.random_alm(7, 7, 1, 0, tag=630))
    with pytest.raises(sht.ShtError) as e:
        plan.alm2map_deriv1(a)
    assert e.value.status == sht.SHT_EINVAL


@pytest.mark.timeout(300)
def test_deriv_gl2047_sampled():
    """Gauss-Legendre 2048 x 4095, lmax 2047, 4 transforms: sampled rings."""
    sht = _sht()
    lmax = 2047
    g = si.gauss_geometry(2048, 4095)
    plan = sht.Plan(sht.Geometry.from_inputs(g), lmax, spin=1, ntrans=4)
    a = si.random_alm(lmax, lmax, 4, 0, tag=640)
    d = to_host(plan.alm2map_deriv1(to_dev(a)))
    rings = np.array([0, 1, 700, 1023, 1024, 2046, 2047])
    trans = [0, 3]
    ref = oracle.deriv_synthesis(g, lmax, lmax, np.ascontiguousarray(a[trans]), rings=rings)
    pix = np.concatenate([np.arange(g.ofs[y], g.ofs[y] + g.nphi[y]) for y in rings])
    assert rel_err(d[trans][..., pix], ref[..., pix]) < TOL64
