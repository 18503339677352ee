"""ctypes binding of libfft3d.so (argument marshalling only).

The library must have been built in-tree (``paper_2006_08435_amd/build.py``
or ``__graft_entry__.build()``).  There is no fallback: if the shared library
is missing, importing the package's GPU entry points raises.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
# FFT3D_LIB_PATH: another build of the same sources (the sanitizer test loads
# one whose host code is address/undefined-behaviour instrumented).
LIB_PATH = os.environ.get("FFT3D_LIB_PATH") or os.path.join(_HERE, "libfft3d.so")

FFT3D_OK = 0
FFT3D_E_INVALID_ARG = -1
FFT3D_E_UNSUPPORTED_SIZE = -2
FFT3D_E_NO_DEVICE = -3
FFT3D_E_ALLOC = -4
FFT3D_E_LAUNCH = -5
FFT3D_E_ALIGNMENT = -6
FFT3D_E_UNSUPPORTED = -7
FFT3D_E_TIMEOUT = -8
FFT3D_E_SCRATCH = -9

FFT3D_FP32 = 0
FFT3D_FP16_SCALED = 1
FFT3D_BF16_SCALED = 2
FFT3D_FORWARD = -1
FFT3D_INVERSE = 1

# Every symbol the C header declares, with (restype, argtypes).
_vp = ctypes.c_void_p
_ci = ctypes.c_int
SIGNATURES = {
    "fft3d_plan": (_vp, [_ci, _ci, _ci, _ci, _ci, _ci]),
    "fft3d_exec": (_ci, [_vp, _vp, _vp, _vp]),
    "fft3d_destroy": (_ci, [_vp]),
    "fft3d_last_error": (_ci, []),
    "fft3d_strerror": (ctypes.c_char_p, [_ci]),
    "fft3d_buffer_bytes": (ctypes.c_size_t, [_vp]),
    "fft3d_plan_describe": (_ci, [_vp, ctypes.c_char_p, ctypes.c_size_t]),
    "fft3d_plan_passes": (_ci, [_vp]),
    "fft3d_plan_check": (_ci, [_vp]),
    "fft3d_plan_set_cutoff": (_ci, [_vp, ctypes.c_double]),
    "fft3d_plan_real": (_vp, [_ci, _ci, _ci, _ci, _ci]),
    "fft3d_apply_potential": (_ci, [_vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "fft3d_density": (_ci, [_vp, _vp, _vp, _vp, _vp, _vp]),
    "fft3d_real_bytes": (ctypes.c_size_t, [_vp]),
    "fft3d_plan_sphere_points": (ctypes.c_longlong, [_vp]),
    "fft3d_sphere_pack": (_ci, [_vp, _vp, _vp, _vp]),
    "fft3d_sphere_unpack": (_ci, [_vp, _vp, _vp, _vp]),
    "fft3d_exec_packed": (_ci, [_vp, _vp, _vp, _vp]),
    "fft3d_quantize": (_ci, [_ci, ctypes.c_long, _ci, _vp, _vp, _vp]),
    "fft3d_dequantize": (_ci, [_ci, ctypes.c_long, _ci, _vp, _vp, _vp]),
    "fft3d_stream_copy": (_ci, [_vp, _vp, ctypes.c_size_t, _vp]),
    "fft3d_plan_many": (_vp, [_ci, _vp, _vp, _vp, _vp, _ci, _ci]),
    "fft3d_exec_many": (_ci, [_vp, _vp, _vp, _vp]),
    "fft3d_plan_set_schedule": (_ci, [_vp, _ci, _ci]),
    "fft3d_plan_set_group_schedule": (_ci, [_vp, _ci, _ci, _ci]),
    "fft3d_plan_tune": (_ci, [_vp]),
    "fft3d_energy_fwd": (_ci, [_vp, _vp, _vp, _vp, _vp, _vp]),
    "fft3d_energy": (_ci, [_vp, _vp, _vp, _vp, _vp, _vp]),
    "fft3d_energy_bwd": (_ci, [_vp, _vp, _ci, _vp, _vp, _vp, _vp]),
    "fft3d_exec_pass": (_ci, [_vp, _ci, _vp, _vp, _vp]),
    "fft3d_energy_noalloc": (_ci, [_ci, _ci, _ci, _ci, _vp, _vp, _vp, _vp, _vp]),
}

_lib = None


class Fft3dError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        self.code = code
        msg = lib().fft3d_strerror(code).decode() if _lib is not None else str(code)
        super().__init__("%s%s (status %d)" % (what + ": " if what else "", msg, code))


def lib():
    """The loaded libfft3d.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libfft3d.so is not built at %s; run __graft_entry__.build() "
                              "(there is no CPU fallback)" % LIB_PATH)
        l = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(l, name)
            fn.restype = res
            fn.argtypes = args
        _lib = l
    return _lib


def check(code: int, what: str = "") -> None:
    if code != FFT3D_OK:
        raise Fft3dError(code, what)
