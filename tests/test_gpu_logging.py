"""SHT_LOG levels 2 and 3 on a real transform: entry-point calls and kernel
launches are reported on stderr, one line each (run in a child process, since
the level is read once per process)."""
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

_SCRIPT = r"""
import torch
import sht_inputs as si
import paper_1303_4945_amd as sht
g = si.gauss_geometry(16, 31)
p = sht.Plan(sht.Geometry.from_inputs(g), 15, spin=2, ntrans=2)
a = torch.from_numpy(si.random_alm(15, 15, 2, 2, tag=3)).cuda()
m = p.alm2map(a)
b = p.map2alm(m)
torch.cuda.synchronize()
print("ok", float((b - a).abs().max()))
"""


def _run(level):
    env = dict(os.environ, SHT_LOG=str(level))
    r = subprocess.run([sys.executable, "-u", "-c", _SCRIPT], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    assert r.stdout.startswith("ok")
    assert float(r.stdout.split()[1]) < 1e-10   # exact Gauss-Legendre round trip
    return [ln for ln in r.stderr.splitlines() if ln.startswith("[sht:")]


def test_log_levels_two_and_three():
    two = _run(2)
    assert any(ln.startswith("[sht:1] plan") and "created" in ln and "spin 2, 2 transforms" in ln for ln in two), two
    assert sum(ln.startswith("[sht:2] sht_execute plan") for ln in two) == 2, two
    assert not any(ln.startswith("[sht:3]") for ln in two)
    three = _run(3)
    launches = [ln for ln in three if ln.startswith("[sht:3] launch")]
    assert any("Legendre synthesis" in ln for ln in launches), three
    assert any("Legendre analysis" in ln for ln in launches), three
    assert any("ring FFT (synthesis)" in ln for ln in launches), three
    assert any("ring FFT (analysis)" in ln for ln in launches), three
