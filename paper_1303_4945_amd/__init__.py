"""Spherical harmonic transforms on AMD MI355X (gfx950).

Thin Python binding of ``libsht.so`` (C ABI in ``include/sht.h``): argument
marshalling only.  Every step of the transforms runs in the library's HIP
kernels; PyTorch supplies device memory and the current stream.  There is no
CPU fallback: if the library is missing, importing this package fails.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsht.so")

SHT_OK, SHT_EINVAL, SHT_ENOMEM, SHT_EDEVICE, SHT_EUNSUPPORTED, SHT_ESTATE = range(6)
FP64, FP32_MFMA = 0, 1
ALM2MAP, MAP2ALM, ALM2MAP_ADJOINT, ALM2MAP_GRAD, MAP2ALM_ADJOINT = 0, 1, 2, 3, 4
ALM2MAP_DERIV1, ALM2MAP_DERIV1_ADJOINT, ALM2MAP_DERIV1_GRAD = 5, 6, 7
_SYNTH_DIRECTIONS = (ALM2MAP, MAP2ALM_ADJOINT, ALM2MAP_DERIV1)
_DERIV_DIRECTIONS = (ALM2MAP_DERIV1, ALM2MAP_DERIV1_ADJOINT, ALM2MAP_DERIV1_GRAD)
ECP_FEJER1, ECP_FEJER2, ECP_CC = 0, 1, 2

_STATUS_NAMES = {1: "SHT_EINVAL", 2: "SHT_ENOMEM", 3: "SHT_EDEVICE", 4: "SHT_EUNSUPPORTED",
                 5: "SHT_ESTATE"}


class ShtError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


if not os.path.exists(LIB_PATH):
    raise ImportError(f"libsht.so not built ({LIB_PATH}); run __graft_entry__.build()")

# torch ships its own HIP runtime under the same soname (libamdhip64.so.7);
# loading torch first makes libsht bind to that one instance, so that device
# pointers and streams from torch are valid inside the library.
import torch  # noqa: E402,F401

_lib = ctypes.CDLL(LIB_PATH)

_vp = ctypes.c_void_p
_dp = ctypes.POINTER(ctypes.c_double)
_i64p = ctypes.POINTER(ctypes.c_int64)


class PlanOpts(ctypes.Structure):
    _fields_ = [("no_polar_skip", ctypes.c_int), ("polar_T", ctypes.c_double),
                ("rescale_bits", ctypes.c_int), ("flush_chunks", ctypes.c_int),
                ("real_harmonics", ctypes.c_int), ("reserved", ctypes.c_int * 7)]


def _sig(name, res, *args):
    f = getattr(_lib, name)
    f.restype = res
    f.argtypes = list(args)
    return f


_sig("sht_last_error", ctypes.c_char_p)
_sig("sht_strerror", ctypes.c_char_p, ctypes.c_int)
_sig("sht_geom_create", ctypes.c_int, ctypes.c_int, _dp, _i64p, _dp, _dp, _i64p, ctypes.c_int64,
     ctypes.POINTER(_vp))
_sig("sht_geom_gauss", ctypes.c_int, ctypes.c_int, ctypes.c_int64, ctypes.c_double,
     ctypes.POINTER(_vp))
_sig("sht_geom_healpix", ctypes.c_int, ctypes.c_int, ctypes.POINTER(_vp))
_sig("sht_geom_ecp", ctypes.c_int, ctypes.c_int, ctypes.c_int64, ctypes.c_int, ctypes.c_double,
     ctypes.POINTER(_vp))
_sig("sht_geom_reduced_gauss", ctypes.c_int, ctypes.c_int, ctypes.c_int64, ctypes.c_int, ctypes.c_int,
     ctypes.c_int, ctypes.c_double, ctypes.POINTER(_vp))
_sig("sht_geom_info", ctypes.c_int, _vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int64))
_sig("sht_geom_rings", ctypes.c_int, _vp, _dp, _i64p, _dp, _dp, _i64p)
_sig("sht_geom_destroy", None, _vp)
_sig("sht_alm_index", ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.c_int)
_sig("sht_nalm", ctypes.c_int64, ctypes.c_int, ctypes.c_int)
_sig("sht_plan_create", ctypes.c_int, _vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
     ctypes.c_int, ctypes.POINTER(PlanOpts), ctypes.POINTER(_vp))
_sig("sht_plan_destroy", None, _vp)
_sig("sht_execute", ctypes.c_int, _vp, ctypes.c_int, _vp, _vp, _vp)
_sig("sht_execute_noalloc", ctypes.c_int, _vp, ctypes.c_int, _vp, _vp, _vp)
_sig("sht_noalloc_capacity", ctypes.c_int, _i64p)
_sig("sht_legendre", ctypes.c_int, _vp, ctypes.c_int, _vp, _vp, _vp)
_sig("sht_ring_fft", ctypes.c_int, _vp, ctypes.c_int, _vp, _vp, _vp)
_sig("sht_plan_flops", ctypes.c_int, _vp, ctypes.c_int, _dp, _dp, _dp)
_sig("sht_plan_info", ctypes.c_int, _vp, _i64p, _i64p)
_sig("sht_memory_stats", ctypes.c_int, _i64p, _i64p)
_sig("sht_batch_create", ctypes.c_int, ctypes.c_int, ctypes.POINTER(_vp), ctypes.POINTER(_vp))
_sig("sht_batch_execute", ctypes.c_int, _vp, ctypes.c_int, ctypes.POINTER(_vp), ctypes.POINTER(_vp), _vp)
_sig("sht_batch_destroy", None, _vp)
_sig("sht_batch_legendre", ctypes.c_int, _vp, ctypes.c_int, ctypes.POINTER(_vp), ctypes.POINTER(_vp), _vp)
_sig("sht_batch_configure", ctypes.c_int, _vp, ctypes.c_int, ctypes.c_int)
_sig("sht_autotune", ctypes.c_int, _vp, ctypes.c_double)


class Tuning(ctypes.Structure):
    _fields_ = [("synth_ncb", ctypes.c_int), ("synth_mblock", ctypes.c_int), ("anal_ncb", ctypes.c_int),
                ("anal_tpw", ctypes.c_int), ("valu", ctypes.c_int), ("reserved", ctypes.c_int * 11)]


_sig("sht_plan_get_tuning", ctypes.c_int, _vp, ctypes.POINTER(Tuning))
_sig("sht_plan_set_tuning", ctypes.c_int, _vp, ctypes.POINTER(Tuning))

lib = _lib


def last_error() -> str:
    return _lib.sht_last_error().decode()


def _check(rc: int):
    if rc != SHT_OK:
        raise ShtError(rc, last_error())


def memory_stats():
    """(live device buffers, their bytes) allocated by the library."""
    n, b = ctypes.c_int64(), ctypes.c_int64()
    _check(_lib.sht_memory_stats(ctypes.byref(n), ctypes.byref(b)))
    return n.value, b.value


def noalloc_capacity() -> int:
    """Bytes of the static workspace of the allocation-free entry point."""
    b = ctypes.c_int64()
    _check(_lib.sht_noalloc_capacity(ctypes.byref(b)))
    return b.value


def nalm(lmax: int, mmax: int) -> int:
    return int(_lib.sht_nalm(lmax, mmax))


def alm_index(lmax: int, l: int, m: int) -> int:
    return int(_lib.sht_alm_index(lmax, l, m))


class Geometry:
    """Iso-latitude ring grid (owned by the library)."""

    def __init__(self, handle):
        self._h = handle
        self._destroy = _lib.sht_geom_destroy
        n = ctypes.c_int()
        npix = ctypes.c_int64()
        _check(_lib.sht_geom_info(self._h, ctypes.byref(n), ctypes.byref(npix)))
        self.nrings = n.value
        self.npix = npix.value

    @classmethod
    def from_arrays(cls, theta, nphi, phi0, weight=None, ofs=None, stride: int = 1):
        theta = np.ascontiguousarray(theta, dtype=np.float64)
        nphi = np.ascontiguousarray(nphi, dtype=np.int64)
        phi0 = np.ascontiguousarray(phi0, dtype=np.float64)
        w = None if weight is None else np.ascontiguousarray(weight, dtype=np.float64)
        o = None if ofs is None else np.ascontiguousarray(ofs, dtype=np.int64)
        h = _vp()
        _check(_lib.sht_geom_create(int(theta.shape[0]), theta.ctypes.data_as(_dp),
                                    nphi.ctypes.data_as(_i64p), phi0.ctypes.data_as(_dp),
                                    None if w is None else w.ctypes.data_as(_dp),
                                    None if o is None else o.ctypes.data_as(_i64p),
                                    int(stride), ctypes.byref(h)))
        return cls(h)

    @classmethod
    def from_inputs(cls, g):
        """From an object with theta/nphi/phi0/weight/ofs/stride attributes."""
        return cls.from_arrays(g.theta, g.nphi, g.phi0, g.weight, g.ofs, g.stride)

    @classmethod
    def gauss(cls, nrings: int, nphi: int, phi0: float = 0.0):
        h = _vp()
        _check(_lib.sht_geom_gauss(nrings, nphi, phi0, ctypes.byref(h)))
        return cls(h)

    @classmethod
    def healpix(cls, nside: int):
        h = _vp()
        _check(_lib.sht_geom_healpix(nside, ctypes.byref(h)))
        return cls(h)

    @classmethod
    def ecp(cls, nrings: int, nphi: int, kind: int = 2, phi0: float = 0.0):
        """Equidistant rings with Fejer-1 (kind 0), Fejer-2 (1) or Clenshaw-Curtis (2) weights."""
        h = _vp()
        _check(_lib.sht_geom_ecp(nrings, nphi, kind, phi0, ctypes.byref(h)))
        return cls(h)

    @classmethod
    def reduced_gauss(cls, nrings: int, nphi_max: int, lmax: int, mmax: int | None = None,
                      spin: int = 0, phi0: float = 0.0):
        """Gauss-Legendre rings with pixel counts thinned by the polar criterion."""
        h = _vp()
        mmax = lmax if mmax is None else mmax
        _check(_lib.sht_geom_reduced_gauss(nrings, nphi_max, lmax, mmax, spin, phi0, ctypes.byref(h)))
        return cls(h)

    def rings(self):
        n = self.nrings
        th, ph, w = np.zeros(n), np.zeros(n), np.zeros(n)
        nphi, ofs = np.zeros(n, dtype=np.int64), np.zeros(n, dtype=np.int64)
        _check(_lib.sht_geom_rings(self._h, th.ctypes.data_as(_dp), nphi.ctypes.data_as(_i64p),
                                   ph.ctypes.data_as(_dp), w.ctypes.data_as(_dp),
                                   ofs.ctypes.data_as(_i64p)))
        return dict(theta=th, nphi=nphi, phi0=ph, weight=w, ofs=ofs)

    def __del__(self):
        # the destroy function is held by the object: at interpreter exit the
        # module's globals may already be gone
        h, fn = getattr(self, "_h", None), getattr(self, "_destroy", None)
        if h and fn is not None:
            fn(h)
            self._h = None


def _stream_handle(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return _vp(s.cuda_stream)


class Plan:
    """A transform plan (geometry, lmax, mmax, spin, ntrans, precision)."""

    def __init__(self, geom: Geometry, lmax: int, mmax: int | None = None, spin: int = 0,
                 ntrans: int = 1, precision: str | int = "fp64", polar: bool = True,
                 polar_T: float | None = None, rescale_bits: int | None = None,
                 flush_chunks: int | None = None, real_harmonics: bool = False):
        mmax = lmax if mmax is None else mmax
        if isinstance(precision, str):
            precision = {"fp64": FP64, "fp32_mfma": FP32_MFMA}[precision]
        o = PlanOpts()
        o.no_polar_skip = 0 if polar else 1
        o.polar_T = float(polar_T or 0.0)
        o.rescale_bits = int(rescale_bits or 0)
        o.flush_chunks = int(flush_chunks or 0)
        o.real_harmonics = 1 if real_harmonics else 0
        h = _vp()
        _check(_lib.sht_plan_create(geom._h, lmax, mmax, spin, ntrans, precision, ctypes.byref(o),
                                    ctypes.byref(h)))
        self._h = h
        self._destroy = _lib.sht_plan_destroy
        self.geom = geom
        self.lmax, self.mmax, self.spin, self.ntrans = lmax, mmax, spin, ntrans
        self.precision = precision
        self.ncomp = 2 if spin else 1
        self.nalm = nalm(lmax, mmax)
        self.npix = geom.npix
        self.nrings = geom.nrings

    # shapes
    @property
    def alm_shape(self):
        return (self.ntrans, self.ncomp, self.nalm, 2)

    @property
    def map_shape(self):
        return (self.ntrans, self.ncomp, self.npix)

    @property
    def deriv_alm_shape(self):
        """Spin-0 coefficients of the derivative directions (spin-1 plans)."""
        return (self.ntrans, 1, self.nalm, 2)

    def out_shape(self, direction):
        if direction in _SYNTH_DIRECTIONS:
            return self.map_shape
        return self.deriv_alm_shape if direction in _DERIV_DIRECTIONS else self.alm_shape

    @property
    def phase_shape(self):
        return (self.ntrans, self.ncomp, self.nrings, self.mmax + 1, 2)

    def _run(self, fn, direction, x, out_shape, stream=None, out=None):
        import torch
        if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == torch.float64):
            raise TypeError("expected a float64 CUDA tensor")
        x = x.contiguous()
        if out is None:
            out = torch.empty(out_shape, dtype=torch.float64, device=x.device)
        _check(fn(self._h, direction, _vp(x.data_ptr()), _vp(out.data_ptr()), _stream_handle(stream)))
        return out

    def alm2map(self, alm, stream=None, out=None):
        return self._run(_lib.sht_execute, ALM2MAP, alm, self.map_shape, stream, out)

    def map2alm(self, maps, stream=None, out=None):
        return self._run(_lib.sht_execute, MAP2ALM, maps, self.alm_shape, stream, out)

    def adjoint(self, maps, stream=None, out=None):
        """Y^T maps (adjoint synthesis: analysis sums with unit weights)."""
        return self._run(_lib.sht_execute, ALM2MAP_ADJOINT, maps, self.alm_shape, stream, out)

    def adjoint_analysis(self, alm, stream=None, out=None):
        """W Y a: synthesis with every ring multiplied by its weight (the adjoint of map2alm)."""
        return self._run(_lib.sht_execute, MAP2ALM_ADJOINT, alm, self.map_shape, stream, out)

    def alm2map_grad(self, grad_maps, stream=None, out=None):
        """dL/d(Re a) + i dL/d(Im a) of a real loss L from dL/dmap (fac_m Y^T g)."""
        return self._run(_lib.sht_execute, ALM2MAP_GRAD, grad_maps, self.alm_shape, stream, out)

    def alm2map_deriv1(self, alm, stream=None, out=None):
        """Maps of df/dtheta and df/(sin theta dphi) from spin-0 a_lm [ntrans][1][nalm][2]
        (Sect. 4.3; the plan must have spin 1)."""
        return self._run(_lib.sht_execute, ALM2MAP_DERIV1, alm, self.map_shape, stream, out)

    def deriv1_adjoint(self, maps, stream=None, out=None):
        """Adjoint of alm2map_deriv1: maps [ntrans][2][npix] -> [ntrans][1][nalm][2]."""
        return self._run(_lib.sht_execute, ALM2MAP_DERIV1_ADJOINT, maps, self.deriv_alm_shape, stream, out)

    def alm2map_deriv1_grad(self, grad_maps, stream=None, out=None):
        """Gradient of a real loss with respect to the a_lm of alm2map_deriv1."""
        return self._run(_lib.sht_execute, ALM2MAP_DERIV1_GRAD, grad_maps, self.deriv_alm_shape, stream, out)

    def execute_noalloc(self, direction, x, stream=None, out=None):
        """sht_execute without any device allocation: the workspace is the
        library's static per-device array (out must then be given by callers
        that cannot allocate)."""
        return self._run(_lib.sht_execute_noalloc, direction, x, self.out_shape(direction), stream, out)

    def legendre_synth(self, alm, stream=None, out=None):
        return self._run(_lib.sht_legendre, ALM2MAP, alm, self.phase_shape, stream, out)

    def legendre_anal(self, phases, stream=None, out=None):
        return self._run(_lib.sht_legendre, MAP2ALM, phases, self.alm_shape, stream, out)

    def ring_synth(self, phases, weights: bool = False, stream=None, out=None):
        d = MAP2ALM_ADJOINT if weights else ALM2MAP
        return self._run(_lib.sht_ring_fft, d, phases, self.map_shape, stream, out)

    def ring_anal(self, maps, weights: bool = True, stream=None, out=None):
        d = MAP2ALM if weights else ALM2MAP_ADJOINT
        return self._run(_lib.sht_ring_fft, d, maps, self.phase_shape, stream, out)

    def flops(self, direction=ALM2MAP):
        """(FP64 flops, FP32 matrix-core flops, minimal HBM bytes) of one Legendre
        step in this direction (see sht_plan_flops)."""
        f, fm, b = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        _check(_lib.sht_plan_flops(self._h, direction, ctypes.byref(f), ctypes.byref(fm), ctypes.byref(b)))
        return f.value, fm.value, b.value

    def info(self):
        n, w = ctypes.c_int64(), ctypes.c_int64()
        _check(_lib.sht_plan_info(self._h, ctypes.byref(n), ctypes.byref(w)))
        return dict(legendre_items=n.value, device_bytes=w.value)

    def autotune(self, budget_seconds: float = 0.1):
        _check(_lib.sht_autotune(self._h, budget_seconds))

    _TUNING_KEYS = ("synth_ncb", "synth_mblock", "anal_ncb", "anal_tpw", "valu")

    def tuning(self) -> dict:
        t = Tuning()
        _check(_lib.sht_plan_get_tuning(self._h, ctypes.byref(t)))
        return {k: getattr(t, k) for k in self._TUNING_KEYS}

    def set_tuning(self, **kw):
        t = Tuning()
        _check(_lib.sht_plan_get_tuning(self._h, ctypes.byref(t)))
        for k, v in kw.items():
            if k not in self._TUNING_KEYS:
                raise KeyError(k)
            setattr(t, k, int(v))
        _check(_lib.sht_plan_set_tuning(self._h, ctypes.byref(t)))

    def __del__(self):
        h, fn = getattr(self, "_h", None), getattr(self, "_destroy", None)
        if h and fn is not None:
            fn(h)
            self._h = None


QUEUE_COST, QUEUE_MPAIRS = 0, 1


class Batch:
    """Several plans (same spin and precision) executed as one unit: the
    Legendre analyses of all plans in one persistent launch over a shared
    queue (plans on the vector path: their own launches); each plan's Legendre synthesis (its die-aware item list) and ring
    FFTs on a stream of its own between a fork and a join; on a non-default
    stream the launches are captured once into a HIP graph per direction
    (captured again when the buffers, the stream or a plan's tuning change)
    and replayed."""

    def __init__(self, plans):
        self.plans = list(plans)
        arr = (_vp * len(self.plans))(*[p._h for p in self.plans])
        h = _vp()
        _check(_lib.sht_batch_create(len(self.plans), arr, ctypes.byref(h)))
        self._h = h
        self._destroy = _lib.sht_batch_destroy

    def execute(self, direction, ins, outs=None, stream=None):
        import torch
        n = len(self.plans)
        if len(ins) != n:
            raise ValueError("one input per plan")
        ins = [x.contiguous() for x in ins]
        for x in ins:
            if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == torch.float64):
                raise TypeError("expected float64 CUDA tensors")
        if outs is None:
            outs = [torch.empty(p.out_shape(direction), dtype=torch.float64, device=x.device)
                    for p, x in zip(self.plans, ins)]
        a_in = (_vp * n)(*[x.data_ptr() for x in ins])
        a_out = (_vp * n)(*[y.data_ptr() for y in outs])
        _check(_lib.sht_batch_execute(self._h, direction, a_in, a_out, _stream_handle(stream)))
        return outs

    def configure(self, queue_order: int = QUEUE_COST, concurrent=True):
        """Queue order and schedule: concurrent True/1 (per-plan chains on
        their own streams), False/0 (one stream) or 2 (persistent synthesis
        over all plans, then per-plan ring FFTs on their own streams)."""
        c = int(concurrent) if not isinstance(concurrent, bool) else (1 if concurrent else 0)
        _check(_lib.sht_batch_configure(self._h, int(queue_order), c))

    def legendre(self, direction, ins, outs, stream=None):
        """Legendre step only of every plan (phases <-> coefficients)."""
        n = len(self.plans)
        a_in = (_vp * n)(*[x.data_ptr() for x in ins])
        a_out = (_vp * n)(*[y.data_ptr() for y in outs])
        _check(_lib.sht_batch_legendre(self._h, direction, a_in, a_out, _stream_handle(stream)))
        return outs

    def alm2map(self, alms, outs=None, stream=None):
        return self.execute(ALM2MAP, alms, outs, stream)

    def map2alm(self, maps, outs=None, stream=None):
        return self.execute(MAP2ALM, maps, outs, stream)

    def __del__(self):
        h, fn = getattr(self, "_h", None), getattr(self, "_destroy", None)
        if h and fn is not None:
            fn(h)
            self._h = None
