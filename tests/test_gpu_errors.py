"""Error paths of the C ABI that need a device: overlapping buffers, failed
device allocations (injected) with no leak, destroyed handles, and a batch
whose member plan was retuned after its launches were captured."""
import ctypes
import os

import numpy as np
import pytest

import sht_inputs as si
from gpu_util import rel_err, to_dev, to_host

pytestmark = pytest.mark.gpu


def _sht():
    import paper_1303_4945_amd as sht
    return sht


def test_overlapping_buffers_rejected():
    import torch
    sht = _sht()
    lmax = 15
    g = si.gauss_geometry(lmax + 1, 2 * lmax + 1)
    p = sht.Plan(sht.Geometry.from_inputs(g), lmax, spin=0, ntrans=1)
    n_alm = int(np.prod(p.alm_shape))
    n_map = int(np.prod(p.map_shape))
    buf = torch.zeros(n_alm + n_map, dtype=torch.float64, device="cuda")
    a = buf[:n_alm].view(p.alm_shape)
    out = buf[n_alm - 1:n_alm - 1 + n_map].view(p.map_shape)   # shares one double with a
    with pytest.raises(sht.ShtError) as e:
        p.alm2map(a, out=out)
    assert e.value.status == sht.SHT_EINVAL and "overlap" in str(e.value)
    ok = buf[n_alm:].view(p.map_shape)
    p.alm2map(a, out=ok)   # adjacent, not overlapping
    # the staged steps check their own byte ranges (phases here)
    ph = torch.zeros(int(np.prod(p.phase_shape)) + 8, dtype=torch.float64, device="cuda")
    with pytest.raises(sht.ShtError) as e:
        p.legendre_anal(ph[:-8].view(p.phase_shape), out=ph[4:4 + n_alm].view(p.alm_shape))
    assert e.value.status == sht.SHT_EINVAL


def test_injected_allocation_failures_leave_no_buffers():
    """SHT_FAULT_INJECT=alloc:N fails the N-th device allocation of a create
    call: every N up to the plan's allocation count gives SHT_ENOMEM and leaves
    the library's live device buffers where they were."""
    sht = _sht()
    lmax = 31
    g = sht.Geometry.from_inputs(si.gauss_geometry(lmax + 1, 2 * lmax + 1))
    base = sht.memory_stats()
    n = 1
    try:
        while True:
            os.environ["SHT_FAULT_INJECT"] = f"alloc:{n}"
            try:
                p = sht.Plan(g, lmax, spin=2, ntrans=2, real_harmonics=True)
            except sht.ShtError as e:
                assert e.status == sht.SHT_ENOMEM, e
                assert sht.memory_stats() == base, n
                n += 1
                assert n < 200
                continue
            break
    finally:
        del os.environ["SHT_FAULT_INJECT"]
    assert n > 10, "the plan made fewer device allocations than expected"
    assert sht.memory_stats()[0] > base[0]
    del p
    assert sht.memory_stats() == base
    # a batch create failing on its first allocation leaves nothing either
    p1 = sht.Plan(g, lmax, spin=0, ntrans=1)
    mid = sht.memory_stats()
    os.environ["SHT_FAULT_INJECT"] = "alloc"
    try:
        with pytest.raises(sht.ShtError) as e:
            sht.Batch([p1])
        assert e.value.status == sht.SHT_ENOMEM
    finally:
        del os.environ["SHT_FAULT_INJECT"]
    assert sht.memory_stats() == mid


def test_schedule_change_failing_allocation_keeps_the_batch():
    """A failed allocation while the persistent synthesis queue is built
    (sht_batch_configure with concurrent 2) gives SHT_ENOMEM, keeps the previous
    schedule and the batch's results, and leaks nothing; switching back to the
    per-plan schedule releases the queue."""
    sht = _sht()
    lmax = 31
    g = sht.Geometry.from_inputs(si.gauss_geometry(lmax + 1, 2 * lmax + 1))
    plans = [sht.Plan(g, lmax, spin=2, ntrans=3) for _ in range(2)]
    a = [to_dev(si.random_alm(lmax, lmax, 3, 2, tag=9 + k)) for k in range(2)]
    b = sht.Batch(plans)
    ref = [to_host(m) for m in b.alm2map(a)]
    base = sht.memory_stats()
    os.environ["SHT_FAULT_INJECT"] = "alloc:2"   # 1: analysis queue, 2: synthesis queue
    try:
        with pytest.raises(sht.ShtError) as e:
            b.configure(sht.QUEUE_COST, 2)
        assert e.value.status == sht.SHT_ENOMEM
    finally:
        del os.environ["SHT_FAULT_INJECT"]
    assert sht.memory_stats() == base
    assert all(np.array_equal(to_host(m), r) for m, r in zip(b.alm2map(a), ref))
    b.configure(sht.QUEUE_COST, 2)
    assert sht.memory_stats()[0] == base[0] + 1   # the synthesis queue
    assert all(np.array_equal(to_host(m), r) for m, r in zip(b.alm2map(a), ref))
    b.configure(sht.QUEUE_COST, 1)
    assert sht.memory_stats() == base


def test_destroyed_plan_rejected_by_execute_and_batch():
    import torch
    sht = _sht()
    lmax = 15
    g = sht.Geometry.from_inputs(si.gauss_geometry(lmax + 1, 2 * lmax + 1))
    p1 = sht.Plan(g, lmax, spin=0, ntrans=1)
    p2 = sht.Plan(g, lmax, spin=0, ntrans=1)
    b = sht.Batch([p1, p2])
    a = to_dev(si.random_alm(lmax, lmax, 1, 0, tag=3))
    b.alm2map([a, a])
    h = p2._h
    sht.lib.sht_plan_destroy(h)
    p2._h = None
    out = torch.empty(p1.map_shape, dtype=torch.float64, device="cuda")
    assert sht.lib.sht_execute(h, 0, ctypes.c_void_p(a.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                               None) == sht.SHT_ESTATE
    with pytest.raises(sht.ShtError) as e:
        b.alm2map([a, a])
    assert e.value.status == sht.SHT_ESTATE
    # a new plan (possibly at the freed address) does not revive the batch
    p3 = sht.Plan(g, lmax, spin=0, ntrans=1)
    with pytest.raises(sht.ShtError) as e:
        b.alm2map([a, a])
    assert e.value.status == sht.SHT_ESTATE
    del p3


def test_batch_graph_recaptured_after_member_retuned(tmp_path):
    """A batch replays its captured graph while buffers and stream stay the
    same; retuning a member plan (new work lists and launch shapes) must
    trigger a new capture.  The tune cache forces the other synthesis
    column-block choice; batch results must equal the plan's own results bit
    for bit before and after."""
    import torch
    sht = _sht()
    lmax = 63
    g = sht.Geometry.from_inputs(si.gauss_geometry(lmax + 1, 2 * lmax + 1))
    p = sht.Plan(g, lmax, spin=2, ntrans=8)
    q = sht.Plan(g, lmax, spin=2, ntrans=2)
    b = sht.Batch([p, q])
    a = [to_dev(si.random_alm(lmax, lmax, 8, 2, tag=11)), to_dev(si.random_alm(lmax, lmax, 2, 2, tag=12))]
    outs = [torch.empty(p.map_shape, dtype=torch.float64, device="cuda"),
            torch.empty(q.map_shape, dtype=torch.float64, device="cuda")]
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        b.alm2map(a, outs=outs, stream=s)
        b.alm2map(a, outs=outs, stream=s)   # graph replay
    s.synchronize()
    ref = to_host(p.alm2map(a[0]))
    assert np.array_equal(to_host(outs[0]), ref)
    before = p.tuning()
    cache = tmp_path / "tune.txt"
    os.environ["SHT_TUNE_CACHE"] = str(cache)
    try:
        # a timed run writes the plan's line; a second line with the other
        # synthesis column-block choice then wins (the last line of a key counts)
        p.autotune(5.0)
        key, val = cache.read_text().strip().splitlines()[-1].rsplit("|", 1)
        other = 1 if p.tuning()["synth_ncb"] == 2 else 2
        fields = dict(kv.split("=") for kv in val.split(","))
        fields["synth_ncb"] = str(other)
        with open(cache, "a") as f:
            f.write(key + "|" + ",".join(f"{k}={v}" for k, v in fields.items()) + "\n")
        p.autotune(0.0)
    finally:
        del os.environ["SHT_TUNE_CACHE"]
    assert p.tuning()["synth_ncb"] == other, "the cached choice was not applied"
    assert p.tuning() != before or before["synth_ncb"] != other
    outs[0].fill_(float("nan"))
    with torch.cuda.stream(s):
        for _ in range(3):
            b.alm2map(a, outs=outs, stream=s)
            s.synchronize()
            assert np.array_equal(to_host(outs[0]), to_host(p.alm2map(a[0])))
    # the matrix-core shapes give the same sums bit for bit; the vector units
    # (a choice the timed run may make) the same terms in another order
    if p.tuning()["valu"] == before["valu"]:
        assert np.array_equal(to_host(outs[0]), ref)
    else:
        assert rel_err(to_host(outs[0]), ref) < 1e-13
