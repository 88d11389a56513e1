"""The allocation-free entry point sht_execute_noalloc (static per-device
workspace) against sht_execute, bit for bit, through the C ABI: two calls in
a row, the second with a smaller input, in every direction family, and the
size limit."""
import ctypes

import numpy as np
import pytest

import sht_inputs as si
from gpu_util import to_dev, to_host

pytestmark = pytest.mark.gpu


def _sht():
    import paper_1303_4945_amd as sht
    return sht


def _call(sht, fn, plan, direction, x, out):
    import torch
    torch.cuda.synchronize()
    rc = fn(plan._h, direction, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()),
            ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    return rc


@pytest.mark.parametrize("spin,real", [(0, False), (2, False), (2, True)])
def test_noalloc_equals_execute_two_calls(spin, real):
    import torch
    sht = _sht()
    cases = [(63, 3), (23, 1)]   # the second call is smaller
    for lmax, ntrans in cases:
        g = si.gauss_geometry(lmax + 1, 2 * lmax + 1)
        p = sht.Plan(sht.Geometry.from_inputs(g), lmax, spin=spin, ntrans=ntrans, real_harmonics=real)
        a = to_dev(si.random_alm(lmax, lmax, ntrans, spin, tag=lmax))
        for direction, x in ((sht.ALM2MAP, a), (sht.MAP2ALM_ADJOINT, a)):
            ref = torch.empty(p.out_shape(direction), dtype=torch.float64, device="cuda")
            got = torch.full_like(ref, float("nan"))
            assert _call(sht, sht.lib.sht_execute, p, direction, x, ref) == sht.SHT_OK
            assert _call(sht, sht.lib.sht_execute_noalloc, p, direction, x, got) == sht.SHT_OK, sht.last_error()
            assert np.array_equal(to_host(got), to_host(ref)), (lmax, direction)
        mp = to_dev(si.random_map(g, ntrans, 2 if spin else 1, tag=lmax + 1))
        for direction in (sht.MAP2ALM, sht.ALM2MAP_ADJOINT, sht.ALM2MAP_GRAD):
            ref = torch.empty(p.out_shape(direction), dtype=torch.float64, device="cuda")
            got = torch.full_like(ref, float("nan"))
            assert _call(sht, sht.lib.sht_execute, p, direction, mp, ref) == sht.SHT_OK
            assert _call(sht, sht.lib.sht_execute_noalloc, p, direction, mp, got) == sht.SHT_OK, sht.last_error()
            assert np.array_equal(to_host(got), to_host(ref)), (lmax, direction)


def test_noalloc_rejects_plans_beyond_the_static_workspace():
    import torch
    sht = _sht()
    cap = sht.noalloc_capacity()
    assert cap == 64 << 20
    # phases of this plan: 8 * 2 * 1024 * 1024 * 16 bytes = 256 MiB > 64 MiB
    lmax = 1023
    g = si.gauss_geometry(lmax + 1, 2 * lmax + 1)
    p = sht.Plan(sht.Geometry.from_inputs(g), lmax, spin=2, ntrans=8)
    a = torch.zeros(p.alm_shape, dtype=torch.float64, device="cuda")
    out = torch.empty(p.map_shape, dtype=torch.float64, device="cuda")
    assert _call(sht, sht.lib.sht_execute_noalloc, p, sht.ALM2MAP, a, out) == sht.SHT_EINVAL
    assert "static scratch" in sht.last_error()
    # a plan that needs the whole array: one scalar transform at lmax 2047 on
    # 2048 rings, 2048 * 2048 * 16 bytes = exactly 64 MiB of phases
    lmax = 2047
    g = si.gauss_geometry(lmax + 1, 2 * lmax + 1)
    p = sht.Plan(sht.Geometry.from_inputs(g), lmax, spin=0, ntrans=1)
    a = to_dev(si.random_alm(lmax, lmax, 1, 0, tag=9))
    ref = p.alm2map(a)
    got = torch.empty_like(ref)
    assert _call(sht, sht.lib.sht_execute_noalloc, p, sht.ALM2MAP, a, got) == sht.SHT_OK
    assert np.array_equal(to_host(got), to_host(ref))
    back_ref = p.map2alm(ref)
    back = torch.empty_like(back_ref)
    assert _call(sht, sht.lib.sht_execute_noalloc, p, sht.MAP2ALM, ref, back) == sht.SHT_OK
    assert np.array_equal(to_host(back), to_host(back_ref))


def test_noalloc_makes_no_device_allocation():
    import torch
    sht = _sht()
    lmax = 31
    g = si.gauss_geometry(lmax + 1, 2 * lmax + 1)
    p = sht.Plan(sht.Geometry.from_inputs(g), lmax, spin=2, ntrans=2)
    a = to_dev(si.random_alm(lmax, lmax, 2, 2, tag=4))
    out = torch.empty(p.map_shape, dtype=torch.float64, device="cuda")
    before = sht.memory_stats()
    assert _call(sht, sht.lib.sht_execute_noalloc, p, sht.ALM2MAP, a, out) == sht.SHT_OK
    assert sht.memory_stats() == before
