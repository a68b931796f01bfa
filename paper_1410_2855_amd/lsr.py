"""Thin ctypes binding of liblsr.so (the HIP C-ABI library).

Argument marshalling only: every step of the round-trip map runs in the HIP
kernels behind the C ABI declared in include/lsr.h.  Functions carry the C
names; device buffers are torch tensors (only their data pointers cross the
boundary) and streams are torch streams.  Importing this module raises if the
library has not been built: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblsr.so")

LSR_OK, LSR_EINVAL, LSR_ENOMEM, LSR_EDEVICE, LSR_EUNSUPPORTED, LSR_ENONFINITE = 0, -1, -2, -3, -4, -5
LSR_PREC_PLAIN, LSR_PREC_FP64TAB, LSR_PREC_FP64 = 0, 1, 2
LSR_AP_NONE, LSR_AP_SUPERGAUSS, LSR_AP_GAUSS, LSR_AP_MASK = 0, 1, 2, 3
LSR_MODEL_B_EULER, LSR_MODEL_B_EXACT, LSR_MODEL_CLASS_A = 0, 1, 2
LSR_MAX_SLICES = 64
LSR_MAX_SHAPES = 2

_STATUS = {0: "LSR_OK", -1: "LSR_EINVAL", -2: "LSR_ENOMEM", -3: "LSR_EDEVICE",
           -4: "LSR_EUNSUPPORTED", -5: "LSR_ENONFINITE"}


class LsrError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("%s: %s" % (_STATUS.get(code, str(code)), msg))
        self.code = code


class lsr_aperture(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("radius", ctypes.c_double),
                ("order", ctypes.c_int), ("mask", ctypes.c_void_p)]


class lsr_diag_out(ctypes.Structure):
    _fields_ = [("energy", ctypes.c_double), ("power_out", ctypes.c_double),
                ("gain_sum", ctypes.c_double), ("aperture_loss", ctypes.c_double),
                ("inv_sum", ctypes.c_double), ("dominant_bin", ctypes.c_int),
                ("nbins", ctypes.c_int), ("radial", ctypes.POINTER(ctypes.c_double))]


_lib = None
_vp = ctypes.c_void_p
_i = ctypes.c_int
_d = ctypes.c_double
_SIGS = {
    "lsr_plan_create": (_i, [ctypes.POINTER(_vp), _i, _d, _d, _d, _d, _d, ctypes.POINTER(lsr_aperture), _i]),
    "lsr_plan_set_gain": (_i, [_vp, _d, _d, _d, _d]),
    "lsr_plan_set_filter": (_i, [_vp, _d]),
    "lsr_plan_set_model": (_i, [_vp, _i]),
    "lsr_plan_set_slices": (_i, [_vp, _i]),
    "lsr_plan_set_roughness": (_i, [_vp, _vp]),
    "lsr_plan_set_transfer": (_i, [_vp, _vp]),
    "lsr_plan_set_fft_plan": (_i, [_vp, _i]),
    "lsr_propagate": (_i, [_vp, _vp, _d, _vp]),
    "lsr_plan_set_stream": (_i, [_vp, _vp]),
    "lsr_roundtrips": (_i, [_vp, _vp, _vp, _i]),
    "lsr_roundtrips_static": (_i, [_i, _d, _d, _d, _d, _d, ctypes.POINTER(lsr_aperture), _d, _d, _d, _d, _i,
                                   _vp, _vp, _i, _vp, _vp]),
    "lsr_sync": (_i, [_vp]),
    "lsr_time_kernels": (_i, [_vp, _vp, _vp, _i, ctypes.POINTER(_d)]),
    "lsr_trace": (_i, [_vp, ctypes.POINTER(_d), _i]),
    "lsr_diag": (_i, [_vp, _vp, _vp, ctypes.POINTER(lsr_diag_out)]),
    "lsr_plan_nbins": (_i, [_vp]),
    "lsr_plan_destroy": (None, [_vp]),
    "lsr_batch_create": (_i, [ctypes.POINTER(_vp), ctypes.POINTER(_vp), _i]),
    "lsr_batch_roundtrips": (_i, [_vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp), _i]),
    "lsr_batch_diag": (_i, [_vp, _i, _vp, _vp, ctypes.POINTER(lsr_diag_out)]),
    "lsr_batch_set_graph_trips": (_i, [_vp, _i]),
    "lsr_batch_prepare": (_i, [_vp, _i]),
    "lsr_batch_test_wait": (_i, [_vp, _i, _i]),
    "lsr_batch_configure": (_i, [_vp, _i, _i, _i, _i, _i, _i, _i, _i, ctypes.POINTER(_i)]),
    "lsr_batch_time_kernels": (_i, [_vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp), _i, ctypes.POINTER(_d)]),
    "lsr_batch_destroy": (None, [_vp]),
    "lsr_autotune": (_i, [_vp, _vp, ctypes.c_char_p]),
    "lsr_last_error": (ctypes.c_char_p, []),
    "lsr_test_fail_alloc": (_i, [_i]),
    "lsr_version": (ctypes.c_char_p, []),
    "lsr_supported": (_i, [_i, _i]),
    "lsr_fft_shape": (_i, [_i, _i, ctypes.POINTER(_i), _i, ctypes.POINTER(_i), ctypes.POINTER(_i)]),
    "lsr_propagator_table": (_i, [_i, _d, _d, _d, ctypes.POINTER(ctypes.c_float)]),
    "lsr_twiddle_table": (_i, [_i, _i, ctypes.POINTER(ctypes.c_float), _i]),
    "lsr_pack_tasks": (_i, [ctypes.POINTER(_i), _i, _i, ctypes.POINTER(_i), _i]),
}


def load(path: str = LIB_PATH):
    """Load liblsr.so (raises if it is missing: build it with build.py)."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise ImportError("liblsr.so is not built (%s); run python -m paper_1410_2855_amd.build" % path)
        lib = ctypes.CDLL(path)
        for name, (res, args) in _SIGS.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib


def exported_symbols():
    return sorted(_SIGS)


def _check(rc: int) -> int:
    if rc < 0:
        raise LsrError(rc, load().lsr_last_error().decode())
    return rc


def _ptr(t) -> int:
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return int(t.data_ptr())


def _stream_handle(stream) -> int:
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)


# ------------------------------------------------------------ C names ----

def lsr_last_error() -> str:
    return load().lsr_last_error().decode()


def lsr_test_fail_alloc(after: int):
    _check(load().lsr_test_fail_alloc(after))


def lsr_version() -> str:
    return load().lsr_version().decode()


def lsr_supported(N: int, prec: int) -> bool:
    return bool(load().lsr_supported(N, prec))


def lsr_fft_shape(N: int, prec: int = LSR_PREC_FP64TAB):
    rad = (ctypes.c_int * 8)()
    lanes, lines = ctypes.c_int(), ctypes.c_int()
    n = _check(load().lsr_fft_shape(N, prec, rad, 8, ctypes.byref(lanes), ctypes.byref(lines)))
    return list(rad[:n]), lanes.value, lines.value


def lsr_propagator_table(N: int, dx: float, lam: float, L: float) -> np.ndarray:
    out = np.zeros(2 * N, dtype=np.float32)
    _check(load().lsr_propagator_table(N, dx, lam, L, out.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
    return out[0::2] + 1j * out[1::2].astype(np.complex64)


def lsr_twiddle_table(N: int, prec: int = LSR_PREC_FP64TAB) -> np.ndarray:
    n = _check(load().lsr_twiddle_table(N, prec, None, 0))
    out = np.zeros(2 * n, dtype=np.float32)
    _check(load().lsr_twiddle_table(N, prec, out.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), n))
    return (out[0::2] + 1j * out[1::2]).astype(np.complex64)


def lsr_pack_tasks(sizes, lag: int = -1) -> np.ndarray:
    s = (ctypes.c_int * len(sizes))(*sizes)
    n = _check(load().lsr_pack_tasks(s, len(sizes), lag, None, 0))
    buf = (ctypes.c_int * (3 * n))()
    _check(load().lsr_pack_tasks(s, len(sizes), lag, buf, n))
    return np.frombuffer(buf, dtype=np.int32).reshape(n, 3).copy()


def lsr_plan_create(N, dx, lam, L, F, R, ap_kind=LSR_AP_SUPERGAUSS, ap_radius=0.0, ap_order=10,
                    ap_mask=None, prec=LSR_PREC_FP64TAB) -> int:
    ap = lsr_aperture(ap_kind, ap_radius, ap_order, _ptr(ap_mask))
    h = ctypes.c_void_p()
    _check(load().lsr_plan_create(ctypes.byref(h), N, dx, lam, L, F, R, ctypes.byref(ap), prec))
    return h.value


def lsr_plan_set_gain(plan, N0, T1, mod_amp=0.0, mod_period=0.0):
    _check(load().lsr_plan_set_gain(plan, N0, T1, mod_amp, mod_period))


def lsr_plan_set_filter(plan, delta: float):
    _check(load().lsr_plan_set_filter(plan, float(delta)))


def lsr_plan_set_model(plan, model: int):
    _check(load().lsr_plan_set_model(plan, int(model)))


def lsr_plan_set_slices(plan, m: int):
    _check(load().lsr_plan_set_slices(plan, int(m)))


def lsr_plan_set_roughness(plan, psi):
    """psi: host N x N float64 roughness phase (rad), or None for a smooth mirror."""
    if psi is None:
        _check(load().lsr_plan_set_roughness(plan, None))
        return
    a = np.ascontiguousarray(psi, dtype=np.float64)
    _check(load().lsr_plan_set_roughness(plan, a.ctypes.data))


def lsr_plan_set_fft_plan(plan, k: int):
    _check(load().lsr_plan_set_fft_plan(plan, int(k)))


def lsr_plan_set_transfer(plan, T):
    """T: host N x N complex transfer function of a general nonlocal step
    (frequency order, row = y frequency), or None for the propagator."""
    if T is None:
        _check(load().lsr_plan_set_transfer(plan, None))
        return
    a = np.ascontiguousarray(T, dtype=np.complex128)
    _check(load().lsr_plan_set_transfer(plan, a.ctypes.data))


def lsr_propagate(plan, E_in, z: float, E_out):
    _check(load().lsr_propagate(plan, _ptr(E_in), float(z), _ptr(E_out)))


def lsr_plan_set_stream(plan, stream):
    _check(load().lsr_plan_set_stream(plan, _stream_handle(stream)))


def lsr_roundtrips(plan, E, Ninv, n_trips: int):
    _check(load().lsr_roundtrips(plan, _ptr(E), _ptr(Ninv), n_trips))


def lsr_roundtrips_static(N, dx, lam, L, F, R, ap, N0, T1, mod_amp, mod_period, model, E, Ninv, n_trips,
                          trace=None, stream=None):
    """The allocation-free form of lsr_roundtrips (no plan): ap is an
    lsr_aperture, trace None or a device float64 tensor of 4 n_trips values."""
    _check(load().lsr_roundtrips_static(N, dx, lam, L, F, R, ctypes.byref(ap), N0, T1, mod_amp, mod_period, model,
                                        _ptr(E), _ptr(Ninv), n_trips, _ptr(trace), _stream_handle(stream)))


def lsr_time_kernels(plan, E, Ninv, n_trips: int):
    """Mean (row-pass ms, column-pass ms) over n_trips event-bracketed trips."""
    ms = (ctypes.c_double * 2)()
    _check(load().lsr_time_kernels(plan, _ptr(E), _ptr(Ninv), n_trips, ms))
    return ms[0], ms[1]


def lsr_sync(plan):
    _check(load().lsr_sync(plan))


def lsr_trace(plan, capacity: int) -> np.ndarray:
    out = np.zeros((max(capacity, 1), 4), dtype=np.float64)
    n = _check(load().lsr_trace(plan, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), capacity))
    return out[:n].copy()


def lsr_plan_nbins(plan) -> int:
    return _check(load().lsr_plan_nbins(plan))


def _diag_result(o: lsr_diag_out, radial: np.ndarray) -> dict:
    return dict(energy=o.energy, power_out=o.power_out, gain_sum=o.gain_sum,
                aperture_loss=o.aperture_loss, inv_sum=o.inv_sum,
                dominant_bin=o.dominant_bin, nbins=o.nbins, radial=radial)


def lsr_diag(plan, E, Ninv) -> dict:
    nb = lsr_plan_nbins(plan)
    radial = np.zeros(nb, dtype=np.float64)
    o = lsr_diag_out()
    o.radial = radial.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    _check(load().lsr_diag(plan, _ptr(E), _ptr(Ninv), ctypes.byref(o)))
    return _diag_result(o, radial)


def lsr_plan_destroy(plan):
    if plan:
        load().lsr_plan_destroy(plan)


def lsr_batch_create(plans) -> int:
    arr = (ctypes.c_void_p * len(plans))(*plans)
    h = ctypes.c_void_p()
    _check(load().lsr_batch_create(ctypes.byref(h), arr, len(plans)))
    return h.value


def lsr_batch_roundtrips(batch, Es, Ns, n_trips: int):
    e = (ctypes.c_void_p * len(Es))(*[_ptr(t) for t in Es])
    n = (ctypes.c_void_p * len(Ns))(*[_ptr(t) for t in Ns])
    _check(load().lsr_batch_roundtrips(batch, e, n, n_trips))


def lsr_batch_diag(batch, idx: int, E, Ninv, nbins: int) -> dict:
    radial = np.zeros(nbins, dtype=np.float64)
    o = lsr_diag_out()
    o.radial = radial.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    _check(load().lsr_batch_diag(batch, idx, _ptr(E), _ptr(Ninv), ctypes.byref(o)))
    return _diag_result(o, radial)


def lsr_batch_set_graph_trips(batch, k: int):
    _check(load().lsr_batch_set_graph_trips(batch, k))


def lsr_batch_prepare(batch, n_trips: int):
    _check(load().lsr_batch_prepare(batch, n_trips))


def lsr_batch_test_wait(batch, extra_need: int, spin_limit: int):
    _check(load().lsr_batch_test_wait(batch, extra_need, spin_limit))


def lsr_batch_configure(batch, engine=-1, variant=-1, wgs_per_cu=-1, chunk=-1, lag=-1, graph_k=-1,
                        merge=-1, shape=-1) -> dict:
    out = (ctypes.c_int * 8)()
    _check(load().lsr_batch_configure(batch, engine, variant, wgs_per_cu, chunk, lag, graph_k, merge, shape, out))
    return dict(zip(("engine", "variant", "wgs_per_cu", "chunk", "lag", "graph_k", "merge", "shape"), out[:]))


def lsr_batch_time_kernels(batch, Es, Ns, n_trips: int):
    """Mean (row-pass ms, column-pass ms, trip ms) over event-bracketed eager trips."""
    e = (ctypes.c_void_p * len(Es))(*[_ptr(t) for t in Es])
    n = (ctypes.c_void_p * len(Ns))(*[_ptr(t) for t in Ns])
    ms = (ctypes.c_double * 3)()
    _check(load().lsr_batch_time_kernels(batch, e, n, n_trips, ms))
    return ms[0], ms[1], ms[2]


def lsr_batch_destroy(batch):
    if batch:
        load().lsr_batch_destroy(batch)


def lsr_autotune(plan=None, batch=None, cache_path: str | None = None):
    _check(load().lsr_autotune(plan, batch, cache_path.encode() if cache_path else None))


# ------------------------------------------------------- convenience ----

class Plan:
    """One cavity plan built from a physical parameter record (inputs.Cavity)."""

    def __init__(self, cav, prec: int = LSR_PREC_FP64TAB, stream=None):
        import torch

        self.cav = cav
        self.prec = prec
        focal = cav.focal if math.isfinite(cav.focal) else 0.0
        self.handle = lsr_plan_create(cav.N, cav.dx, cav.lam, cav.L, focal, cav.R,
                                      ap_kind=cav.ap_kind, ap_radius=cav.ap_radius,
                                      ap_order=cav.ap_order, prec=prec)
        try:
            lsr_plan_set_gain(self.handle, cav.N0, cav.T1, cav.mod_amp, cav.mod_period)
            if getattr(cav, "filter_delta", 0.0):
                lsr_plan_set_filter(self.handle, cav.filter_delta)
            if getattr(cav, "model", 0):
                lsr_plan_set_model(self.handle, cav.model)
            if getattr(cav, "slices", 1) != 1:
                lsr_plan_set_slices(self.handle, cav.slices)
            if getattr(cav, "rough_rms", 0.0):
                from .inputs import rough_field
                lsr_plan_set_roughness(self.handle, rough_field(cav))
            lsr_plan_set_stream(self.handle, stream if stream is not None else torch.cuda.current_stream())
        except BaseException:
            # a failed set-up leaves no plan behind
            self.close()
            raise

    @property
    def cdtype(self):
        import torch
        return torch.complex128 if self.prec == LSR_PREC_FP64 else torch.complex64

    @property
    def rdtype(self):
        import torch
        return torch.float64 if self.prec == LSR_PREC_FP64 else torch.float32

    def state(self, E0: np.ndarray, N0: np.ndarray, device="cuda"):
        """Device copies (E, Ninv) of a host state in this plan's precision."""
        import torch
        e = torch.from_numpy(np.ascontiguousarray(E0)).to(device=device, dtype=self.cdtype).contiguous()
        n = torch.from_numpy(np.ascontiguousarray(N0)).to(device=device, dtype=self.rdtype).contiguous()
        return e, n

    def roundtrips(self, E, Ninv, n_trips: int):
        lsr_roundtrips(self.handle, E, Ninv, n_trips)

    def sync(self):
        lsr_sync(self.handle)

    def trace(self, capacity: int) -> np.ndarray:
        return lsr_trace(self.handle, capacity)

    def propagate(self, E, z: float, out=None):
        """The field E propagated freely over z metres (new tensor unless out)."""
        import torch
        out = torch.empty_like(E) if out is None else out
        lsr_propagate(self.handle, E, z, out)
        return out

    def diag(self, E, Ninv) -> dict:
        return lsr_diag(self.handle, E, Ninv)

    def close(self):
        if self.handle:
            lsr_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
