"""Differentiation form: the backward of alm2map (adjoint synthesis with the
real-field factor) against central differences, the dot-product identity and
the CPU oracle's transpose."""
import numpy as np
import pytest

import oracle
import sht_inputs as si
from gpu_util import rel_err, to_dev, to_host

pytestmark = pytest.mark.gpu


def _mods():
    import torch
    import paper_1303_4945_amd as sht
    from paper_1303_4945_amd import autograd
    return torch, sht, autograd


def _loss_and_grad(plan, a, d):
    torch, sht, ag = _mods()
    x = a.clone().requires_grad_(True)
    mp = ag.alm2map(x, plan)
    loss = 0.5 * torch.sum((mp - d) ** 2)
    loss.backward()
    return loss.item(), x.grad.detach()


def _fd_entries(plan1, a, d, grad, entries, h):
    """Central differences of L = 0.5||Y a - d||^2 at the given (t, c, i, reim)
    entries, evaluated stably: L+ - L- = 0.5 sum (p+ - p-)(p+ + p- - 2d)."""
    torch, sht, _ = _mods()
    out = []
    for (t, c, i, ri) in entries:
        ap = a[t:t + 1].clone()
        am = a[t:t + 1].clone()
        ap[0, c, i, ri] += h
        am[0, c, i, ri] -= h
        pp = plan1.alm2map(ap)
        pm = plan1.alm2map(am)
        dl = 0.5 * torch.sum((pp - pm) * (pp + pm - 2 * d[t:t + 1]))
        out.append(dl.item() / (2 * h))
    got = np.array([grad[t, c, i, ri].item() for (t, c, i, ri) in entries])
    return np.array(out), got


def _entries(rng, ntrans, ncomp, lmax, n, spin):
    ls, ms = si.lm_arrays(lmax, lmax)
    ok = np.nonzero(ls >= spin)[0]
    res = []
    for _ in range(n):
        i = int(rng.choice(ok))
        ri = int(rng.integers(0, 2)) if ms[i] > 0 else 0
        res.append((int(rng.integers(0, ntrans)), int(rng.integers(0, ncomp)), i, ri))
    return res


@pytest.mark.parametrize("spin,grid", [(0, ("healpix", 8)), (2, ("gauss", 20, 39))])
def test_backward_vs_central_differences_small(spin, grid):
    torch, sht, _ = _mods()
    g = si.make_geometry(grid)
    lmax = 19 if spin else 23
    ncomp = 2 if spin else 1
    geom = sht.Geometry.from_inputs(g)
    plan = sht.Plan(geom, lmax, spin=spin, ntrans=3)
    plan1 = sht.Plan(geom, lmax, spin=spin, ntrans=1)
    a = to_dev(si.random_alm(lmax, lmax, 3, spin, tag=51))
    d = to_dev(si.random_map(g, 3, ncomp, tag=52))
    _, grad = _loss_and_grad(plan, a, d)
    rng = np.random.default_rng(5)
    ent = _entries(rng, 3, ncomp, lmax, 24, spin)
    fd, got = _fd_entries(plan1, a, d, grad, ent, 1e-3)
    assert np.max(np.abs(fd - got)) <= 1e-8 * max(1.0, np.max(np.abs(got)))


@pytest.mark.parametrize("spin", [0, 2])
def test_grad_is_fac_times_oracle_transpose(spin):
    """alm2map_grad(g) = fac_m Y^T g with Y^T from the CPU oracle."""
    torch, sht, _ = _mods()
    g = si.healpix_geometry(8)
    lmax = 20
    ncomp = 2 if spin else 1
    plan = sht.Plan(sht.Geometry.from_inputs(g), lmax, spin=spin, ntrans=2)
    gm = si.random_map(g, 2, ncomp, tag=61)
    got = to_host(plan.alm2map_grad(to_dev(gm)))
    ref = oracle.adjoint_synthesis(g, lmax, lmax, spin, gm)
    _, ms = si.lm_arrays(lmax, lmax)
    ref = ref * np.where(ms == 0, 1.0, 2.0)[None, None, :, None]
    assert rel_err(got, ref) < 1e-11


def test_dot_product_identity():
    """<Y a, g> = <a, grad> for the real pairing of (re, im) slots."""
    torch, sht, _ = _mods()
    g = si.gauss_geometry(40, 79)
    plan = sht.Plan(sht.Geometry.from_inputs(g), 39, spin=2, ntrans=2)
    a = si.random_alm(39, 39, 2, 2, spectrum="unit", tag=71)
    gm = si.random_map(g, 2, 2, tag=72)
    ya = to_host(plan.alm2map(to_dev(a)))
    gr = to_host(plan.alm2map_grad(to_dev(gm)))
    lhs = float(np.sum(ya * gm))
    rhs = float(np.sum(a * gr))
    assert abs(lhs - rhs) <= 1e-11 * max(1.0, abs(lhs))


def test_hp2048_workload_finite_differences():
    """Loss 0.5||alm2map(a) - d||^2 on HEALPix Nside=2048, lmax=4095, 8 maps;
    d = alm2map(a_true) + white noise 0.1; central differences on 32 random
    coefficients with h = 1e-3 rms(a)."""
    torch, sht, _ = _mods()
    g = si.healpix_geometry(2048)
    lmax = 4095
    geom = sht.Geometry.from_inputs(g)
    plan = sht.Plan(geom, lmax, spin=0, ntrans=8)
    plan1 = sht.Plan(geom, lmax, spin=0, ntrans=1)
    a_true = to_dev(si.random_alm(lmax, lmax, 8, 0, tag=81))
    noise = torch.from_numpy(si.random_map(g, 8, 1, sigma=0.1, tag=82)).cuda()
    d = plan.alm2map(a_true) + noise
    a = a_true + to_dev(si.random_alm(lmax, lmax, 8, 0, tag=83))
    _, grad = _loss_and_grad(plan, a, d)
    h = 1e-3 * float(torch.sqrt(torch.mean(a ** 2)))
    rng = np.random.default_rng(2048)
    ent = _entries(rng, 8, 1, lmax, 32, 0)
    fd, got = _fd_entries(plan1, a, d, grad, ent, h)
    err = np.max(np.abs(fd - got)) / np.max(np.abs(got))
    assert err < 1e-6, err
    # the backward against the oracle: fac_m Y^T (alm2map(a) - d) on sampled m
    # of two of the maps
    resid = to_host(plan.alm2map(a) - d)[[0, 7]]
    ms = np.array([0, 1, 2, 2048, 4094, 4095])
    ref = oracle.adjoint_synthesis(g, lmax, lmax, 0, resid, ms=ms)
    ref = ref * np.where(si.lm_arrays(lmax, lmax)[1] == 0, 1.0, 2.0)[None, None, :, None]
    sel = np.concatenate([np.arange(m * (2 * lmax + 1 - m) // 2 + m, m * (2 * lmax + 1 - m) // 2 + lmax + 1)
                          for m in ms])
    gh = to_host(grad)[[0, 7]]
    assert rel_err(gh[:, :, sel], ref[:, :, sel]) < 1e-11
