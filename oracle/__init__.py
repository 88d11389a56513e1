"""CPU reference for the spherical harmonic transforms -- test infrastructure.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may use
this package; the GPU library never imports, links or calls it.

It wraps ``sht_oracle.c`` (plain C99 + OpenMP, long double arithmetic with an
extended exponent), which evaluates the paper's definitions directly:
Eq. 10 + Eq. 11 for lambda, Eq. 4 and a direct per-ring DFT (Eq. 3) for
synthesis, a direct per-ring DFT (Eq. 6) and Eq. 5 for analysis.  See the
header comment of ``sht_oracle.c`` for conventions and layouts.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sht_oracle.c")
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_i64p = ctypes.POINTER(ctypes.c_int64)
_ip = ctypes.POINTER(ctypes.c_int)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no fast-math: IEEE semantics throughout)."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is None:
        # SHT_ORACLE_SO: an alternative build of the same source (the sanitizer
        # test loads an AddressSanitizer build this way)
        so = os.environ.get("SHT_ORACLE_SO")
        if not so:
            so = _SO
            if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
                build()
        lib = ctypes.CDLL(so)
        lib.oracle_lambda.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                      ctypes.c_double, _dp]
        lib.oracle_lambda.restype = ctypes.c_int
        lib.oracle_wigner_d.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                        ctypes.c_double]
        lib.oracle_wigner_d.restype = ctypes.c_double
        lib.oracle_synthesis.argtypes = [ctypes.c_int, _dp, _i64p, _dp, _i64p, ctypes.c_int64,
                                         ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                         _dp, _dp, ctypes.c_int, _ip, _dp]
        lib.oracle_synthesis.restype = ctypes.c_int
        lib.oracle_analysis.argtypes = [ctypes.c_int, _dp, _i64p, _dp, _dp, _i64p,
                                        ctypes.c_int64, ctypes.c_int, ctypes.c_int,
                                        ctypes.c_int, ctypes.c_int, _dp, _dp, ctypes.c_int,
                                        _ip, _dp]
        lib.oracle_analysis.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a, typ):
    return a.ctypes.data_as(typ) if a is not None else None


def lam(lmax: int, m: int, s: int, theta: float) -> np.ndarray:
    """s_lambda_lm(theta) for l = 0..lmax (zero below max(|m|,|s|))."""
    out = np.zeros(lmax + 1)
    rc = _load().oracle_lambda(lmax, m, s, float(theta), _ptr(out, _dp))
    if rc:
        raise ValueError(f"oracle_lambda rc={rc}")
    return out


def wigner_d(j: int, mp: int, mm: int, beta: float) -> float:
    return float(_load().oracle_wigner_d(j, mp, mm, float(beta)))


def _geom_arrays(geom):
    return (np.ascontiguousarray(geom.theta, dtype=np.float64),
            np.ascontiguousarray(geom.nphi, dtype=np.int64),
            np.ascontiguousarray(geom.phi0, dtype=np.float64),
            np.ascontiguousarray(geom.weight, dtype=np.float64),
            np.ascontiguousarray(geom.ofs, dtype=np.int64))


def synthesis(geom, lmax: int, mmax: int, spin: int, alm: np.ndarray, rings=None,
              want_phases: bool = False):
    """alm float64 [ntrans][ncomp][nalm][2] -> map [ntrans][ncomp][npix]
    (only the pixels of ``rings`` are filled when a subset is given).
    With want_phases also returns F [ntrans][ncomp][nrings][mmax+1][2]."""
    th, nph, p0, _, ofs = _geom_arrays(geom)
    alm = np.ascontiguousarray(alm, dtype=np.float64)
    ntrans, ncomp = alm.shape[0], alm.shape[1]
    mp = np.zeros((ntrans, ncomp, geom.npix))
    F = np.zeros((ntrans, ncomp, geom.nrings, mmax + 1, 2)) if want_phases else None
    sel = None if rings is None else np.ascontiguousarray(rings, dtype=np.int32)
    nsel = 0 if sel is None else int(sel.shape[0])
    rc = _load().oracle_synthesis(geom.nrings, _ptr(th, _dp), _ptr(nph, _i64p), _ptr(p0, _dp),
                                  _ptr(ofs, _i64p), int(geom.stride), lmax, mmax, spin,
                                  ntrans, _ptr(alm, _dp), _ptr(mp, _dp), nsel,
                                  _ptr(sel, _ip), _ptr(F, _dp))
    if rc:
        raise RuntimeError(f"oracle_synthesis rc={rc}")
    return (mp, F) if want_phases else mp


def analysis(geom, lmax: int, mmax: int, spin: int, maps: np.ndarray, weight=None, ms=None,
             want_phases: bool = False):
    """maps float64 [ntrans][ncomp][npix] -> alm [ntrans][ncomp][nalm][2]
    (only the m in ``ms`` are filled when a subset is given).  ``weight``
    overrides the geometry's ring weights (ones = adjoint synthesis).
    With want_phases also returns G [ntrans][ncomp][nrings][mmax+1][2]."""
    th, nph, p0, w, ofs = _geom_arrays(geom)
    if weight is not None:
        w = np.ascontiguousarray(np.broadcast_to(weight, th.shape), dtype=np.float64)
    maps = np.ascontiguousarray(maps, dtype=np.float64)
    ntrans, ncomp = maps.shape[0], maps.shape[1]
    n = (mmax + 1) * (lmax + 1) - (mmax * (mmax + 1)) // 2
    alm = np.zeros((ntrans, ncomp, n, 2))
    G = np.zeros((ntrans, ncomp, geom.nrings, mmax + 1, 2)) if want_phases else None
    sel = None if ms is None else np.ascontiguousarray(ms, dtype=np.int32)
    nsel = 0 if sel is None else int(sel.shape[0])
    rc = _load().oracle_analysis(geom.nrings, _ptr(th, _dp), _ptr(nph, _i64p), _ptr(p0, _dp),
                                 _ptr(w, _dp), _ptr(ofs, _i64p), int(geom.stride), lmax, mmax,
                                 spin, ntrans, _ptr(maps, _dp), _ptr(alm, _dp), nsel,
                                 _ptr(sel, _ip), _ptr(G, _dp))
    if rc:
        raise RuntimeError(f"oracle_analysis rc={rc}")
    return (alm, G) if want_phases else alm


def adjoint_synthesis(geom, lmax: int, mmax: int, spin: int, maps: np.ndarray, ms=None):
    """Y^T applied to maps: the analysis sums with all weights equal to one."""
    return analysis(geom, lmax, mmax, spin, maps, weight=1.0, ms=ms)


def _degrees(lmax: int, mmax: int) -> np.ndarray:
    """l of every stored coefficient, m-major order (m = 0 .. mmax, l = m .. lmax)."""
    return np.concatenate([np.arange(m, lmax + 1) for m in range(mmax + 1)]).astype(np.float64)


def deriv_synthesis(geom, lmax: int, mmax: int, alm: np.ndarray, rings=None):
    """Maps of the first derivatives of a real scalar field (Sect. 4.3).

    alm float64 [ntrans][1][nalm][2] (spin 0) -> [ntrans][2][npix] holding
    df/dtheta and df/(sin theta dphi).  Following the paper's remark that this
    is a spin-1 transform: the spin-raising operator maps Y_lm to
    sqrt(l (l + 1)) times the spin-1 harmonic, and with the convention
    Q + iU = sum 1_a 1_Y, 1_a = -(E + iB), the spin-1 synthesis of
    E = sqrt(l (l + 1)) a, B = 0 is Q = df/dtheta, U = df/(sin theta dphi).
    """
    alm = np.asarray(alm, dtype=np.float64)
    k = np.sqrt(_degrees(lmax, mmax) * (_degrees(lmax, mmax) + 1.0))
    e = np.zeros((alm.shape[0], 2) + alm.shape[2:])
    e[:, 0] = alm[:, 0] * k[:, None]
    return synthesis(geom, lmax, mmax, 1, e, rings=rings)


def deriv_adjoint(geom, lmax: int, mmax: int, maps: np.ndarray, ms=None):
    """Adjoint of deriv_synthesis: maps [ntrans][2][npix] -> [ntrans][1][nalm][2],
    sqrt(l (l + 1)) times the E part of the spin-1 Y^T."""
    eb = adjoint_synthesis(geom, lmax, mmax, 1, maps, ms=ms)
    k = np.sqrt(_degrees(lmax, mmax) * (_degrees(lmax, mmax) + 1.0))
    return eb[:, :1] * k[None, None, :, None]


# ---------------------------------------------------------------- real harmonics
# Real spherical harmonics (Sect. 4.5 refers their definition to an external
# appendix; this reading): R_l0 = Y_l0 and, for m > 0, R_lm = sqrt(2) Re Y_lm,
# R_l,-m = sqrt(2) Im Y_lm.  A real field f = sum r_lm R_lm then has the complex
# coefficients a_l0 = r_l0, a_lm = (r_lm - i r_l,-m) / sqrt(2) (m > 0), and
# r_l,-m is stored in the slot of Im a_lm.

def _m_of_index(lmax: int, mmax: int) -> np.ndarray:
    return np.concatenate([np.full(lmax + 1 - m, m) for m in range(mmax + 1)])


def real_to_complex(lmax: int, mmax: int, r: np.ndarray) -> np.ndarray:
    """[.., nalm, 2] real-harmonic coefficients -> complex a_lm (same layout)."""
    r = np.asarray(r, dtype=np.float64)
    mpos = _m_of_index(lmax, mmax) > 0
    a = np.zeros_like(r)
    a[..., ~mpos, 0] = r[..., ~mpos, 0]
    a[..., mpos, 0] = r[..., mpos, 0] / np.sqrt(2.0)
    a[..., mpos, 1] = -r[..., mpos, 1] / np.sqrt(2.0)
    return a


def complex_to_real(lmax: int, mmax: int, a: np.ndarray) -> np.ndarray:
    """Inverse of real_to_complex (Im a_l0 is dropped)."""
    a = np.asarray(a, dtype=np.float64)
    mpos = _m_of_index(lmax, mmax) > 0
    r = np.zeros_like(a)
    r[..., ~mpos, 0] = a[..., ~mpos, 0]
    r[..., mpos, 0] = np.sqrt(2.0) * a[..., mpos, 0]
    r[..., mpos, 1] = -np.sqrt(2.0) * a[..., mpos, 1]
    return r


def synthesis_real(geom, lmax: int, mmax: int, spin: int, r: np.ndarray, rings=None):
    """Synthesis from real-harmonic coefficients."""
    return synthesis(geom, lmax, mmax, spin, real_to_complex(lmax, mmax, r), rings=rings)


def analysis_real(geom, lmax: int, mmax: int, spin: int, maps: np.ndarray, ms=None):
    """Analysis returning real-harmonic coefficients."""
    return complex_to_real(lmax, mmax, analysis(geom, lmax, mmax, spin, maps, ms=ms))


def adjoint_synthesis_real(geom, lmax: int, mmax: int, spin: int, maps: np.ndarray, ms=None):
    """Transpose of synthesis_real: the chain rule through real_to_complex turns
    fac_m Y^T x into sqrt(2) (Re, -Im) of Y^T x for m > 0, i.e. complex_to_real
    of the plain Y^T."""
    return complex_to_real(lmax, mmax, adjoint_synthesis(geom, lmax, mmax, spin, maps, ms=ms))
