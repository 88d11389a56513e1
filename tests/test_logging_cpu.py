"""Diagnostics of the library: the SHT_LOG levels on stderr and the roctx
ranges linked around the entry points (host side only; no GPU needed)."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

_SCRIPT = r"""
import paper_1303_4945_amd as sht
g = sht.Geometry.gauss(8, 15)
print("npix", g.npix)
try:
    sht.Geometry.gauss(0, 15)
except sht.ShtError as e:
    print("rejected", e.status)
del g
"""


def _run(level):
    env = dict(os.environ)
    env.pop("SHT_LOG", None)
    if level is not None:
        env["SHT_LOG"] = str(level)
    r = subprocess.run([sys.executable, "-c", _SCRIPT], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 0, r.stderr
    assert "npix 120" in r.stdout and "rejected" in r.stdout
    return [ln for ln in r.stderr.splitlines() if ln.startswith("[sht:")]


def test_log_off_by_default():
    assert _run(None) == []
    assert _run(0) == []


def test_log_level_one_reports_handles_and_errors():
    lines = _run(1)
    assert any("geometry" in ln and "created: 8 rings, 120 pixels" in ln for ln in lines), lines
    assert any(ln.startswith("[sht:1] error: nrings 0") for ln in lines), lines
    assert any("geometry destroyed (8 rings)" in ln for ln in lines), lines
    assert all(ln.startswith("[sht:1]") for ln in lines)


def test_log_level_clamped():
    assert _run(7) == _run(3)


def test_entry_points_carry_roctx_ranges():
    nm = shutil.which("nm")
    if nm is None:
        pytest.skip("nm not available")
    import paper_1303_4945_amd as sht
    out = subprocess.run([nm, "-D", "--undefined-only", sht.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    assert "roctxRangePushA" in out and "roctxRangePop" in out
