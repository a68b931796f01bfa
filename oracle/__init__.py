"""FP64 CPU oracle of the split-step round-trip map (test infrastructure).

Only the test suite, the package smoke check and the CPU-baseline leg of the
benchmark may import this module.  It wraps ``liborc.so`` (plain C, built by
:func:`build`) with ctypes and never touches the GPU library: the two share no
code.  Every function takes and returns NumPy arrays.

The method follows the paper's Introduction, Eq. (1), and Sec. 2.2,
Eqs. (11)-(12), with the diffraction step taken as the operator exponent of
Sec. 2.3, Eq. (25); the C source states each reading it makes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "orc.c")
_LIB = os.path.join(_HERE, "liborc.so")
_lib = None


# ORC_SANITIZE=1 builds and loads a separate copy instrumented with
# AddressSanitizer and UndefinedBehaviorSanitizer (any finding aborts); the
# process must then preload the ASan runtime.  The arithmetic is unchanged.
_SANITIZE = os.environ.get("ORC_SANITIZE") == "1"
if _SANITIZE:
    _LIB = os.path.join(_HERE, "liborc_san.so")


def build(force: bool = False) -> str:
    """Compile ``orc.c`` into ``liborc.so`` with strict IEEE FP64 flags."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < max(
        os.path.getmtime(_SRC), os.path.getmtime(os.path.join(_HERE, "orc.h"))
    ):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = [
            "gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fno-fast-math",
            "-ffp-contract=off", "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm",
        ]
        if _SANITIZE:
            cmd[1:1] = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


class _Params(ctypes.Structure):
    _fields_ = [
        ("N", ctypes.c_int),
        ("dx", ctypes.c_double),
        ("lam", ctypes.c_double),
        ("L", ctypes.c_double),
        ("focal", ctypes.c_double),
        ("R", ctypes.c_double),
        ("ap_kind", ctypes.c_int),
        ("ap_radius", ctypes.c_double),
        ("ap_order", ctypes.c_int),
        ("ap_mask", ctypes.POINTER(ctypes.c_double)),
        ("N0", ctypes.c_double),
        ("T1", ctypes.c_double),
        ("mod_amp", ctypes.c_double),
        ("mod_period", ctypes.c_double),
        ("filter_delta", ctypes.c_double),
        ("model", ctypes.c_int),
        ("slices", ctypes.c_int),
        ("rough", ctypes.POINTER(ctypes.c_double)),
        ("transfer", ctypes.POINTER(ctypes.c_double)),
    ]


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        lib.orc_fft1d.argtypes = [dp, ctypes.c_int, ctypes.c_int]
        lib.orc_dft_brute1d.argtypes = [dp, dp, ctypes.c_int, ctypes.c_int]
        lib.orc_fft2.argtypes = [dp, ctypes.c_int, ctypes.c_int]
        lib.orc_dft_brute2d.argtypes = [dp, dp, ctypes.c_int, ctypes.c_int]
        lib.orc_run.argtypes = [ctypes.POINTER(_Params), dp, dp, ctypes.c_int, dp]
        lib.orc_nbins.argtypes = [ctypes.c_int]
        lib.orc_spectrum.argtypes = [ctypes.POINTER(_Params), dp, dp, dp, ctypes.c_int]
        lib.orc_propagate.argtypes = [ctypes.POINTER(_Params), dp, ctypes.c_double]
        for f in ("orc_fft1d", "orc_dft_brute1d", "orc_fft2", "orc_dft_brute2d",
                  "orc_run", "orc_nbins", "orc_spectrum", "orc_propagate"):
            getattr(lib, f).restype = ctypes.c_int
        _lib = lib
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _c128(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.complex128)


@dataclass
class CavityParams:
    """Physical parameters of one cavity (SI units; gain in log units)."""

    N: int
    dx: float
    lam: float
    L: float
    R: float
    N0: float
    T1: float
    focal: float = float("inf")
    ap_kind: int = 1
    ap_radius: float = 0.0
    ap_order: int = 10
    ap_mask: np.ndarray | None = None
    mod_amp: float = 0.0
    mod_period: float = 0.0
    filter_delta: float = 0.0   # > 0: Gaussian renormalization-group filter instead of Fresnel
    model: int = 0              # 0 B class (Euler), 1 B class (exact over a trip), 2 class A
    slices: int = 1             # thin gain sheets per iterate (inversion holds one N x N map each)
    rough: np.ndarray | None = None  # N x N roughness phase psi (rad) of Eq. (12), or None
    transfer: np.ndarray | None = None  # N x N complex transfer function of a general nonlocal step
                                        # (Eq. (10)), FFT order, row = y frequency; or None

    def _c(self):
        p = _Params()
        p.N, p.dx, p.lam, p.L = self.N, self.dx, self.lam, self.L
        p.focal = 0.0 if not np.isfinite(self.focal) else self.focal
        p.R, p.ap_kind, p.ap_radius, p.ap_order = self.R, self.ap_kind, self.ap_radius, self.ap_order
        p.N0, p.T1, p.mod_amp, p.mod_period = self.N0, self.T1, self.mod_amp, self.mod_period
        p.filter_delta = self.filter_delta
        p.model = self.model
        p.slices = self.slices
        keep = []
        if self.ap_kind == 3:
            keep.append(np.ascontiguousarray(self.ap_mask, dtype=np.float64).reshape(self.N, self.N))
            p.ap_mask = _dp(keep[-1])
        if self.rough is not None:
            keep.append(np.ascontiguousarray(self.rough, dtype=np.float64).reshape(self.N, self.N))
            p.rough = _dp(keep[-1])
        if self.transfer is not None:
            keep.append(np.ascontiguousarray(self.transfer, dtype=np.complex128).reshape(self.N, self.N))
            p.transfer = _dp(keep[-1].view(np.float64))
        return p, keep


def fft1d(x, inverse: bool = False) -> np.ndarray:
    a = _c128(x).copy()
    if _load().orc_fft1d(_dp(a.view(np.float64)), a.size, int(inverse)) != 0:
        raise ValueError("orc_fft1d: unsupported length %d" % a.size)
    return a


def dft_brute1d(x, inverse: bool = False) -> np.ndarray:
    a = _c128(x)
    out = np.empty_like(a)
    if _load().orc_dft_brute1d(_dp(a.view(np.float64)), _dp(out.view(np.float64)),
                               a.size, int(inverse)) != 0:
        raise ValueError("orc_dft_brute1d failed")
    return out


def fft2(x, inverse: bool = False) -> np.ndarray:
    a = _c128(x).copy()
    n = a.shape[0]
    assert a.shape == (n, n)
    if _load().orc_fft2(_dp(a.view(np.float64)), n, int(inverse)) != 0:
        raise ValueError("orc_fft2: unsupported size %d" % n)
    return a


def dft_brute2d(x, inverse: bool = False) -> np.ndarray:
    a = _c128(x)
    n = a.shape[0]
    out = np.empty_like(a)
    if _load().orc_dft_brute2d(_dp(a.view(np.float64)), _dp(out.view(np.float64)),
                               n, int(inverse)) != 0:
        raise ValueError("orc_dft_brute2d failed")
    return out


def run(params: CavityParams, E, Ninv, n_trips: int):
    """Advance (E, Ninv) by ``n_trips`` iterates; returns (E, Ninv, trace).

    ``trace`` has shape (n_trips, 4): raw sums S1 = sum|E|^2,
    S2 = sum|A|^2|E|^2, S3 = sum|A|^2 e^N |E|^2, S4 = sum N of each trip's
    incoming state.  With ``params.slices`` = m > 1, ``Ninv`` holds the m
    sheets' inversions, shape (m, N, N), and the sums are those of sheet 0.
    """
    n = params.N
    m = max(int(params.slices), 1)
    e = _c128(E).reshape(n, n).copy()
    ninv = np.ascontiguousarray(Ninv, dtype=np.float64).reshape((m, n, n) if m > 1 else (n, n)).copy()
    trace = np.zeros((max(n_trips, 0), 4), dtype=np.float64)
    p, keep = params._c()
    rc = _load().orc_run(ctypes.byref(p), _dp(e.view(np.float64)), _dp(ninv),
                         int(n_trips), _dp(trace) if n_trips > 0 else None)
    del keep
    if rc != 0:
        raise ValueError("orc_run: invalid parameters")
    return e, ninv, trace


def propagate(params: CavityParams, E, z: float) -> np.ndarray:
    """E propagated freely over z metres (no local step)."""
    n = params.N
    e = _c128(E).reshape(n, n).copy()
    p, keep = params._c()
    rc = _load().orc_propagate(ctypes.byref(p), _dp(e.view(np.float64)), float(z))
    del keep
    if rc != 0:
        raise ValueError("orc_propagate: invalid arguments")
    return e


def nbins(N: int) -> int:
    return int(_load().orc_nbins(int(N)))


def spectrum(params: CavityParams, E, Ninv):
    """Radial far-field spectrum of G = sqrt(R) A e^{N/2} E; returns (radial, dominant_bin)."""
    n = params.N
    e = _c128(E).reshape(n, n)
    ninv = np.ascontiguousarray(Ninv, dtype=np.float64).reshape(n, n)
    nb = nbins(n)
    radial = np.zeros(nb, dtype=np.float64)
    p, keep = params._c()
    k = _load().orc_spectrum(ctypes.byref(p), _dp(e.view(np.float64)), _dp(ninv), _dp(radial), nb)
    del keep
    if k < 0:
        raise ValueError("orc_spectrum failed")
    return radial, int(k)
