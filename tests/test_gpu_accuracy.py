"""The accuracy experiment of Sect. 5 (evaluation of SHT pairs) on the GPU path.

Coefficients with real and imaginary parts uniform on [-1, 1) (Im a_l0 = 0) go
through a synthesis onto a reduced Gauss-Legendre grid and an analysis back; the
errors of the pair are the relative rms error over all (l, m) and the largest
absolute error of one coefficient.  The paper reports that both stay near the
double-precision limit at low band limits, the rms error growing about linearly
with lmax and the largest error about as lmax^(3/2), for spin 0 and likewise
for spins 2 and 37.  Its values are plotted, not printed, so the gates take
those growth laws with a constant of one unit roundoff u = 2^-53:
eps_rms <= u (lmax + 1) and eps_max <= u (lmax + 1)^(3/2).  The vector kernels
(one transform) and the matrix-core kernels (several) are both covered; the FP32
matrix-core form is held to its own relative accuracy of 1e-6."""
import math

import numpy as np
import pytest

import sht_inputs as si
from gpu_util import to_dev, to_host

pytestmark = pytest.mark.gpu

U = 2.0 ** -53


def _sht():
    import paper_1303_4945_amd as sht
    return sht


def _pair_errors(a, back):
    """Relative rms error over every stored coefficient and the largest absolute
    error, both as defined for the SHT-pair test."""
    d = back - a
    rms = math.sqrt(float(np.sum(d * d)) / float(np.sum(a * a)))
    mx = float(np.max(np.hypot(d[..., 0], d[..., 1])))
    return rms, mx


@pytest.mark.parametrize("spin,lmax,ntrans", [
    (0, 63, 1), (0, 255, 1), (0, 1023, 1), (0, 4095, 1), (0, 4095, 4),
    (2, 255, 1), (2, 1023, 1), (2, 4095, 1), (2, 2047, 4),
    (37, 255, 1), (37, 1023, 1),
])
def test_sht_pair_errors(spin, lmax, ntrans):
    sht = _sht()
    geom = sht.Geometry.reduced_gauss(lmax + 1, 2 * lmax + 2, lmax, lmax, spin, 0.0)
    plan = sht.Plan(geom, lmax, spin=spin, ntrans=ntrans)
    a = si.random_alm(lmax, lmax, ntrans, spin, spectrum="uniform", tag=900 + spin)
    print(f"\nspin {spin} lmax {lmax} transforms {ntrans}, tuning {plan.tuning()}", flush=True)
    back = to_host(plan.map2alm(plan.alm2map(to_dev(a))))
    rms, mx = _pair_errors(a, back)
    print(f"eps_rms {rms:.3e} ({rms / (U * (lmax + 1)):.3f} u (lmax+1)), "
          f"eps_max {mx:.3e} ({mx / (U * (lmax + 1) ** 1.5):.3f} u (lmax+1)^1.5)")
    assert rms <= U * (lmax + 1)
    assert mx <= U * (lmax + 1) ** 1.5


@pytest.mark.parametrize("spin,lmax,ntrans", [(0, 2047, 8), (2, 1023, 16), (2, 4095, 4)])
def test_sht_pair_errors_fp32_form(spin, lmax, ntrans):
    """The same experiment in the FP32 matrix-core form: relative rms error of the
    pair within 1e-6, the form's accuracy target (FP32 products of FP64 values,
    FP64 accumulation carried every few chunks)."""
    sht = _sht()
    geom = sht.Geometry.reduced_gauss(lmax + 1, 2 * lmax + 2, lmax, lmax, spin, 0.0)
    plan = sht.Plan(geom, lmax, spin=spin, ntrans=ntrans, precision="fp32_mfma")
    a = si.random_alm(lmax, lmax, ntrans, spin, spectrum="uniform", tag=950 + spin)
    print(f"\nfp32 form: spin {spin} lmax {lmax} transforms {ntrans}", flush=True)
    back = to_host(plan.map2alm(plan.alm2map(to_dev(a))))
    rms, mx = _pair_errors(a, back)
    print(f"eps_rms {rms:.3e}, eps_max {mx:.3e}")
    assert rms <= 1e-6
