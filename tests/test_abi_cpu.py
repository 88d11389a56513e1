"""Host-side checks of the C ABI: exports, geometry helpers, indexing and
argument validation (no GPU needed; no transform is computed here)."""
import math
import os
import re

import numpy as np
import pytest

import sht_inputs as si

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _sht():
    import paper_1303_4945_amd as sht
    return sht


def test_exports_every_declared_symbol():
    sht = _sht()
    hdr = open(os.path.join(ROOT, "include", "sht.h")).read()
    names = sorted(set(re.findall(
        r"^(?:int|void|int64_t|const char)\s*\*?\s*(sht_[a-z_0-9]+)\s*\(", hdr, re.M)))
    assert len(names) >= 20
    for n in names:
        assert hasattr(sht.lib, n), n


def test_alm_indexing():
    sht = _sht()
    for lmax, mmax in [(0, 0), (7, 7), (10, 3), (4095, 4095)]:
        assert sht.nalm(lmax, mmax) == si.nalm(lmax, mmax)
        ls, ms = si.lm_arrays(lmax, mmax)
        if lmax < 20:
            for i, (l, m) in enumerate(zip(ls, ms)):
                assert sht.alm_index(lmax, int(l), int(m)) == i
    assert sht.nalm(3, 5) == 0


@pytest.mark.parametrize("n", [1, 2, 5, 64, 255, 1024])
def test_gauss_geometry_matches_inputs(n):
    sht = _sht()
    g = sht.Geometry.gauss(n, 2 * n + 1, 0.25)
    r = g.rings()
    ref = si.gauss_geometry(n, 2 * n + 1, 0.25)
    assert np.max(np.abs(r["theta"] - ref.theta)) < 4e-15
    assert np.max(np.abs(r["weight"] / ref.weight - 1)) < 1e-13
    assert np.all(r["nphi"] == ref.nphi) and np.all(r["ofs"] == ref.ofs)
    assert abs(np.sum(r["weight"] * r["nphi"]) - 4 * math.pi) < 1e-12


@pytest.mark.parametrize("nside", [1, 2, 16, 1024])
def test_healpix_geometry_matches_inputs(nside):
    sht = _sht()
    g = sht.Geometry.healpix(nside)
    r = g.rings()
    ref = si.healpix_geometry(nside)
    assert g.npix == 12 * nside * nside == ref.npix
    assert np.array_equal(r["nphi"], ref.nphi)
    assert np.max(np.abs(r["theta"] - ref.theta)) < 1e-15
    assert np.max(np.abs(r["phi0"] - ref.phi0)) < 1e-15
    assert np.allclose(r["weight"], 4 * math.pi / g.npix, rtol=1e-15)


def test_geometry_validation():
    sht = _sht()
    th = np.array([0.5, 1.0])
    nphi = np.array([4, 4])
    p0 = np.zeros(2)
    with pytest.raises(sht.ShtError) as e:
        sht.Geometry.from_arrays(np.array([0.5, 4.0]), nphi, p0)
    assert e.value.status == sht.SHT_EINVAL
    with pytest.raises(sht.ShtError) as e:
        sht.Geometry.from_arrays(th, np.array([4, 0]), p0)
    assert e.value.status == sht.SHT_EINVAL
    with pytest.raises(sht.ShtError) as e:
        sht.Geometry.from_arrays(th, nphi, p0, stride=0)
    assert e.value.status == sht.SHT_EINVAL
    g = sht.Geometry.from_arrays(th, nphi, p0, ofs=np.array([0, 10]), stride=2)
    assert g.npix == 10 + 3 * 2 + 1


def test_plan_argument_validation_before_device():
    sht = _sht()
    g = sht.Geometry.gauss(8, 17)
    cases = [dict(lmax=-1), dict(lmax=7, mmax=9), dict(lmax=7, ntrans=0),
             dict(lmax=1, spin=2), dict(lmax=7, spin=-1), dict(lmax=3, spin=4),
             dict(lmax=7, precision=7), dict(lmax=7, rescale_bits=10)]
    for kw in cases:
        with pytest.raises(sht.ShtError) as e:
            sht.Plan(g, **kw)
        assert e.value.status == sht.SHT_EINVAL, kw


def test_invalid_handles():
    sht = _sht()
    assert sht.lib.sht_geom_info(None, None, None) == sht.SHT_ESTATE
    assert sht.lib.sht_execute(None, 0, None, None, None) == sht.SHT_ESTATE
    assert sht.lib.sht_strerror(sht.SHT_ENOMEM).decode() == "out of memory"


def test_no_device_reports_edevice():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    sht = _sht()
    g = sht.Geometry.gauss(8, 17)
    with pytest.raises(sht.ShtError) as e:
        sht.Plan(g, 7)
    assert e.value.status == sht.SHT_EDEVICE


def test_plan_opts_layout_matches_header(tmp_path):
    """The ctypes mirror of sht_plan_opts has the C layout of include/sht.h."""
    import ctypes
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    sht = _sht()
    fields = [f for f, _ in sht.PlanOpts._fields_]
    src = tmp_path / "layout.c"
    src.write_text("#include <stdio.h>\n#include <stddef.h>\n#include \"sht.h\"\nint main(void) {\n"
                   "  printf(\"%zu\\n\", sizeof(sht_plan_opts));\n"
                   + "".join(f"  printf(\"%zu\\n\", offsetof(sht_plan_opts, {f}));\n" for f in fields)
                   + "  return 0;\n}\n")
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)])
    out = [int(v) for v in subprocess.check_output([str(exe)]).split()]
    assert out[0] == ctypes.sizeof(sht.PlanOpts)
    assert out[1:] == [getattr(sht.PlanOpts, f).offset for f in fields]


def test_destroyed_and_foreign_handles_are_rejected():
    """Handles are looked up in the library's registry before they are read:
    a destroyed geometry, a pointer that never was a handle and a handle of
    the wrong kind all give SHT_ESTATE (and no read of freed memory)."""
    import ctypes
    sht = _sht()
    h = ctypes.c_void_p()
    assert sht.lib.sht_geom_gauss(8, 17, 0.0, ctypes.byref(h)) == sht.SHT_OK
    n = ctypes.c_int()
    assert sht.lib.sht_geom_info(h, ctypes.byref(n), None) == sht.SHT_OK and n.value == 8
    sht.lib.sht_geom_destroy(h)
    assert sht.lib.sht_geom_info(h, ctypes.byref(n), None) == sht.SHT_ESTATE
    sht.lib.sht_geom_destroy(h)   # a second destroy is a no-op
    junk = (ctypes.c_double * 16)()
    assert sht.lib.sht_geom_info(ctypes.cast(junk, ctypes.c_void_p), None, None) == sht.SHT_ESTATE
    g = sht.Geometry.gauss(4, 9)
    # a geometry handle passed where a plan is expected
    assert sht.lib.sht_execute(g._h, 0, None, None, None) == sht.SHT_ESTATE
    f = ctypes.c_double()
    assert sht.lib.sht_plan_flops(g._h, 0, ctypes.byref(f), None, None) == sht.SHT_ESTATE
    assert sht.lib.sht_batch_execute(g._h, 0, None, None, None) == sht.SHT_ESTATE


def test_memory_stats_without_device():
    sht = _sht()
    n, b = sht.memory_stats()
    assert n >= 0 and b >= 0
