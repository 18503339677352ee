"""FP64 CPU oracle for the complex 3D DFT -- test infrastructure only.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product library never loads it and
shares no code with it: the arithmetic lives in ``oracle/oracle.c`` (plain C,
double precision), built here with gcc into ``oracle/liboracle.so``.

Functions (each follows a passage of the paper, Ramaswami et al., "Efficient
Ab-Initio Molecular Dynamic Simulations by Offloading Fast Fourier
Transformations to FPGAs"):

* ``dft3d_naive`` -- Section II, Eq. (1) term by term (W_N = exp(-2 pi i/N)).
* ``fft3d`` -- Section II: 1D transforms along x, then y, then z, each a
  recursive mixed-radix (5, 3, 2) FFT.  ``order`` permutes the axes.
* ``fft1d`` -- the same 1D recursion on a single sequence.
* ``q16_encode`` / ``q16_decode`` -- the scaled 16-bit storage format of the
  reduced-precision form (the paper's low-precision motivation, Section I and
  Section III closing paragraph): per-row power-of-two exponent and an IEEE
  binary16 or bfloat16 payload.
* ``energy`` -- the plane-wave local-potential energy E = sum V |IFFT(c)|^2
  and its gradient (the operator evaluation that Section I names as the
  reason 3D FFTs sit on the critical path).

Sign convention: ``sign=-1`` is Eq. (1); ``sign=+1`` is the unnormalised
inverse.  Arrays are numpy, C order [batch][z][y][x], complex128.
"""
from __future__ import annotations

import contextlib
import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

FMT_FP16 = 1
FMT_BF16 = 2


def build(force: bool = False) -> str:
    """Compile oracle.c with gcc (IEEE double, OpenMP) into liboracle.so."""
    if (not force and os.path.exists(_LIB)
            and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC)):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
           "-fno-fast-math", "-ffp-contract=off", _SRC, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


def _bind(lib):
    dp = ctypes.POINTER(ctypes.c_double)
    fp = ctypes.POINTER(ctypes.c_float)
    u16 = ctypes.POINTER(ctypes.c_uint16)
    i8 = ctypes.POINTER(ctypes.c_int8)
    ci = ctypes.c_int
    lib.oracle_dft3d_naive.argtypes = [ci, ci, ci, ci, ci, dp, dp]
    lib.oracle_fft3d.argtypes = [ci, ci, ci, ci, ci, dp, dp]
    lib.oracle_fft3d_order.argtypes = [ci, ci, ci, ci, ci, dp, dp, ctypes.POINTER(ci)]
    lib.oracle_fft1d.argtypes = [ci, ci, dp, dp]
    lib.oracle_set_threads.argtypes = [ci]
    lib.oracle_set_threads.restype = None
    lib.oracle_max_threads.restype = ci
    lib.oracle_round_fp16.argtypes = [ctypes.c_double]
    lib.oracle_round_fp16.restype = ctypes.c_uint16
    lib.oracle_round_bf16.argtypes = [ctypes.c_double]
    lib.oracle_round_bf16.restype = ctypes.c_uint16
    lib.oracle_fp16_value.argtypes = [ctypes.c_uint16]
    lib.oracle_fp16_value.restype = ctypes.c_double
    lib.oracle_bf16_value.argtypes = [ctypes.c_uint16]
    lib.oracle_bf16_value.restype = ctypes.c_double
    lib.oracle_q16_encode.argtypes = [ci, ctypes.c_long, ci, fp, u16, i8]
    lib.oracle_q16_decode.argtypes = [ci, ctypes.c_long, ci, u16, i8, dp]
    lib.oracle_energy.argtypes = [ci, ci, ci, ci, dp, dp, dp, dp, dp]
    lib.oracle_apply_potential.argtypes = [ci, ci, ci, ci, dp, dp, dp]
    lib.oracle_density.argtypes = [ci, ci, ci, ci, dp, dp, dp]
    lib.oracle_r2c3d.argtypes = [ci, ci, ci, ci, dp, dp]
    lib.oracle_c2r3d.argtypes = [ci, ci, ci, ci, dp, dp]
    return lib


def _load():
    global _lib
    with _lock:
        if _lib is None:
            # FFT3D_ORACLE_LIB: another build of oracle.c (the sanitizer test
            # runs the pins against an address/undefined-behaviour
            # instrumented one)
            alt = os.environ.get("FFT3D_ORACLE_LIB")
            if not alt:
                build()
            _lib = _bind(ctypes.CDLL(alt or _LIB))
        return _lib


def build_variant(source: str, out_path: str) -> str:
    """Compile a (modified) copy of oracle.c's text into ``out_path``.

    Used only by the mutation tests, which plant a mistake in the oracle and
    check that its pins catch it."""
    src = out_path + ".c"
    with open(src, "w") as f:
        f.write(source)
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
           "-fno-fast-math", "-ffp-contract=off", src, "-o", out_path, "-lm"]
    subprocess.run(cmd, check=True)
    return out_path


@contextlib.contextmanager
def variant(lib_path: str):
    """Route every function of this module to another build of oracle.c."""
    global _lib
    old = _load()
    with _lock:
        _lib = _bind(ctypes.CDLL(lib_path))
    try:
        yield
    finally:
        with _lock:
            _lib = old


def source_text() -> str:
    with open(_SRC) as f:
        return f.read()


def _ptr(a, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def _shape3(a):
    a = np.ascontiguousarray(a, dtype=np.complex128)
    if a.ndim == 3:
        return a[None], True
    if a.ndim == 4:
        return a, False
    raise ValueError("expected [z,y,x] or [batch,z,y,x], got %r" % (a.shape,))


def _check(rc):
    if rc != 0:
        raise RuntimeError("oracle call failed with code %d" % rc)


def set_threads(n: int) -> None:
    _load().oracle_set_threads(int(n))


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def dft3d_naive(a, sign: int = -1) -> np.ndarray:
    """Eq. (1) summed term by term; a is [z,y,x] or [b,z,y,x]."""
    lib = _load()
    x, squeeze = _shape3(a)
    b, nz, ny, nx = x.shape
    out = np.empty_like(x)
    _check(lib.oracle_dft3d_naive(nx, ny, nz, b, int(sign),
                                  _ptr(x, ctypes.c_double), _ptr(out, ctypes.c_double)))
    return out[0] if squeeze else out


def fft3d(a, sign: int = -1, order=(0, 1, 2)) -> np.ndarray:
    """Separable FFT: 1D passes along the axes in ``order`` (0=x, 1=y, 2=z)."""
    lib = _load()
    x, squeeze = _shape3(a)
    b, nz, ny, nx = x.shape
    out = np.empty_like(x)
    o = (ctypes.c_int * 3)(*[int(v) for v in order])
    _check(lib.oracle_fft3d_order(nx, ny, nz, b, int(sign),
                                  _ptr(x, ctypes.c_double), _ptr(out, ctypes.c_double), o))
    return out[0] if squeeze else out


def apply_potential(c, V) -> np.ndarray:
    """forward(V * inverse(c)) per grid (unnormalised both ways)."""
    lib = _load()
    x, squeeze = _shape3(c)
    b, nz, ny, nx = x.shape
    v = np.ascontiguousarray(V, dtype=np.float64)
    if v.shape != (nz, ny, nx):
        raise ValueError("V must be [z, y, x] of the grid shape")
    out = np.empty_like(x)
    _check(lib.oracle_apply_potential(nx, ny, nz, b, _ptr(x, ctypes.c_double), _ptr(v, ctypes.c_double),
                                      _ptr(out, ctypes.c_double)))
    return out[0] if squeeze else out


def density(c, occ) -> np.ndarray:
    """rho = sum_n occ[n] |inverse(c_n)|^2, a real [z, y, x] grid."""
    lib = _load()
    x, _ = _shape3(c)
    b, nz, ny, nx = x.shape
    f = np.ascontiguousarray(occ, dtype=np.float64).ravel()
    if f.size != b:
        raise ValueError("one occupation per orbital")
    rho = np.empty((nz, ny, nx), np.float64)
    _check(lib.oracle_density(nx, ny, nz, b, _ptr(x, ctypes.c_double), _ptr(f, ctypes.c_double),
                              _ptr(rho, ctypes.c_double)))
    return rho


def r2c3d(f) -> np.ndarray:
    """Half spectrum [.., z, y, x/2+1] of a real grid [.., z, y, x] (x even)."""
    lib = _load()
    x = np.ascontiguousarray(f, dtype=np.float64)
    squeeze = x.ndim == 3
    if squeeze:
        x = x[None]
    b, nz, ny, nx = x.shape
    out = np.empty((b, nz, ny, nx // 2 + 1), np.complex128)
    _check(lib.oracle_r2c3d(nx, ny, nz, b, _ptr(x, ctypes.c_double), _ptr(out, ctypes.c_double)))
    return out[0] if squeeze else out


def c2r3d(h, nx: int) -> np.ndarray:
    """Unnormalised real inverse of a half spectrum [.., z, y, nx/2+1]."""
    lib = _load()
    x = np.ascontiguousarray(h, dtype=np.complex128)
    squeeze = x.ndim == 3
    if squeeze:
        x = x[None]
    b, nz, ny, hh = x.shape
    if hh != nx // 2 + 1:
        raise ValueError("half spectrum width %d does not match nx=%d" % (hh, nx))
    out = np.empty((b, nz, ny, nx), np.float64)
    _check(lib.oracle_c2r3d(nx, ny, nz, b, _ptr(x, ctypes.c_double), _ptr(out, ctypes.c_double)))
    return out[0] if squeeze else out


def fft1d(a, sign: int = -1) -> np.ndarray:
    lib = _load()
    x = np.ascontiguousarray(a, dtype=np.complex128).ravel()
    out = np.empty_like(x)
    _check(lib.oracle_fft1d(x.size, int(sign), _ptr(x, ctypes.c_double),
                            _ptr(out, ctypes.c_double)))
    return out


def round_fp16(v: float) -> int:
    return int(_load().oracle_round_fp16(float(v)))


def round_bf16(v: float) -> int:
    return int(_load().oracle_round_bf16(float(v)))


def fp16_value(h: int) -> float:
    return float(_load().oracle_fp16_value(int(h)))


def bf16_value(h: int) -> float:
    return float(_load().oracle_bf16_value(int(h)))


def q16_encode(a, fmt: int):
    """Scaled 16-bit encoding of complex64 rows.

    ``a``: complex64 array whose last axis is the row (x).  Returns
    ``(payload, exps)``: uint16 array of shape a.shape + (2,) holding (re, im)
    bit patterns, and int8 exponents of shape a.shape[:-1].
    """
    lib = _load()
    a = np.ascontiguousarray(a, dtype=np.complex64)
    row_len = a.shape[-1]
    rows = a.size // row_len
    f = a.view(np.float32)
    payload = np.empty(a.shape + (2,), dtype=np.uint16)
    exps = np.empty(a.shape[:-1], dtype=np.int8)
    _check(lib.oracle_q16_encode(int(fmt), rows, row_len, _ptr(f, ctypes.c_float),
                                 _ptr(payload, ctypes.c_uint16), _ptr(exps, ctypes.c_int8)))
    return payload, exps


def q16_decode(payload, exps, fmt: int) -> np.ndarray:
    """Exact value (payload * 2^e) of a scaled 16-bit array, as complex128."""
    lib = _load()
    payload = np.ascontiguousarray(payload, dtype=np.uint16)
    exps = np.ascontiguousarray(exps, dtype=np.int8)
    shape = payload.shape[:-1]
    row_len = shape[-1]
    rows = int(np.prod(shape[:-1], dtype=np.int64))
    out = np.empty(shape, dtype=np.complex128)
    _check(lib.oracle_q16_decode(int(fmt), rows, row_len, _ptr(payload, ctypes.c_uint16),
                                 _ptr(exps, ctypes.c_int8), _ptr(out, ctypes.c_double)))
    return out


def energy(c, V, want_psi: bool = False, want_grad: bool = True):
    """E = sum_n sum_r V |psi_n|^2 with psi_n = unnormalised inverse of c_n.

    Returns (E, psi or None, grad or None); grad = dE/dRe c + i dE/dIm c.
    """
    lib = _load()
    x, squeeze = _shape3(c)
    b, nz, ny, nx = x.shape
    Vd = np.ascontiguousarray(V, dtype=np.float64)
    if Vd.shape != (nz, ny, nx):
        raise ValueError("V must have shape %r" % ((nz, ny, nx),))
    E = ctypes.c_double(0.0)
    psi = np.empty_like(x) if want_psi else None
    grad = np.empty_like(x) if want_grad else None
    null = ctypes.POINTER(ctypes.c_double)()
    _check(lib.oracle_energy(nx, ny, nz, b, _ptr(x, ctypes.c_double), _ptr(Vd, ctypes.c_double),
                             ctypes.byref(E),
                             _ptr(psi, ctypes.c_double) if psi is not None else null,
                             _ptr(grad, ctypes.c_double) if grad is not None else null))
    if squeeze:
        psi = psi[0] if psi is not None else None
        grad = grad[0] if grad is not None else None
    return E.value, psi, grad
