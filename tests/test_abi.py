"""The C ABI: exported symbols and host-side argument checks (CPU, no GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER_DIR = os.path.join(ROOT, "include")


def _lib():
    from paper_2006_08435_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    return _lib


def declared_functions():
    names = set()
    for fn in os.listdir(HEADER_DIR):
        if fn.endswith(".h"):
            text = open(os.path.join(HEADER_DIR, fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(fft3d_[a-z0-9_]+)\s*\(", text))
    return names


def test_every_declared_symbol_is_exported():
    L = _lib()
    names = declared_functions()
    assert "fft3d_plan" in names and "fft3d_exec" in names
    raw = ctypes.CDLL(L.LIB_PATH)
    for n in sorted(names):
        assert hasattr(raw, n), "missing export " + n
    # and the binding knows every declared function
    assert names <= set(L.SIGNATURES), names - set(L.SIGNATURES)


def test_no_undeclared_c_exports():
    """Every unmangled symbol the library defines is a declared entry point."""
    import subprocess
    L = _lib()
    out = subprocess.run(["nm", "-D", "--defined-only", L.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    plain = {ln.split()[-1] for ln in out.splitlines() if ln.split() and ln.split()[1] in "TtWw"}
    plain = {n for n in plain if not n.startswith("_")}
    assert plain == declared_functions(), plain ^ declared_functions()


@pytest.mark.parametrize("args,code", [
    ((0, 16, 16, 1, 0, -1), -1), ((-1, 16, 16, 1, 0, -1), -1), ((16, 16, 16, 0, 0, -1), -1),
    ((16, 16, 16, -3, 0, -1), -1), ((16, 16, 16, 1, 3, -1), -1), ((16, 16, 16, 1, -1, -1), -1),
    ((16, 16, 16, 1, 0, 0), -1), ((16, 16, 16, 1, 0, 2), -1),
    ((7, 16, 16, 1, 0, -1), -2), ((16, 11, 16, 1, 0, -1), -2), ((16, 16, 129, 1, 0, -1), -2),
    ((1024, 16, 16, 1, 0, -1), -2), ((14, 16, 16, 1, 0, -1), -2), ((16, 16, 514, 1, 0, -1), -2),
    ((16, 16, 1000, 1, 0, -1), -2), ((256, 256, 256, 1, 1, -1), -7), ((16, 512, 16, 1, 2, 1), -7),
])
def test_plan_rejects_bad_arguments(args, code):
    L = _lib()
    lib = L.lib()
    assert not lib.fft3d_plan(*args)
    assert lib.fft3d_last_error() == code


def test_null_handles():
    lib = _lib().lib()
    assert lib.fft3d_destroy(None) == 0
    assert lib.fft3d_buffer_bytes(None) == 0
    assert lib.fft3d_exec(None, None, None, None) == -1
    assert lib.fft3d_plan_describe(None, None, 0) == -1
    assert lib.fft3d_plan_set_cutoff(None, 10.0) == -1
    assert lib.fft3d_plan_sphere_points(None) == -1
    assert lib.fft3d_sphere_pack(None, None, None, None) == -1
    assert lib.fft3d_sphere_unpack(None, None, None, None) == -1
    assert lib.fft3d_exec_packed(None, None, None, None) == -1
    assert lib.fft3d_real_bytes(None) == 0
    assert lib.fft3d_apply_potential(None, None, None, None, None, None, None) == -1
    assert lib.fft3d_density(None, None, None, None, None, None) == -1
    assert lib.fft3d_energy(None, None, None, None, None, None) == -1
    assert lib.fft3d_energy_noalloc(16, 16, 16, 1, None, None, None, None, None) == -1


def test_noalloc_argument_checks():
    """The no-allocation entry point checks its arguments before any HIP call
    (the pointers below are never dereferenced)."""
    lib = _lib().lib()
    f = lib.fft3d_energy_noalloc
    assert f(16, 16, 16, 0, 4096, 4096, 4096, 4096, None) == -1
    assert f(16, 16, 16, 1, 4104, 4096, 4096, 4096, None) == -6
    assert f(16, 16, 16, 1, 4096, 4096, 4096, 4100, None) == -6
    assert f(14, 14, 16, 1, 4096, 4096, 4096, 4096, None) == -2
    assert f(16, 8, 16, 1, 4096, 4096, 4096, 4096, None) == -7
    assert f(128, 128, 1, 511, 4096, 4096, 4096, 4096, None) == -9


def test_stream_copy_argument_checks():
    """The measurement copy checks its arguments before any HIP call."""
    lib = _lib().lib()
    assert lib.fft3d_stream_copy(None, None, 16, None) == -1
    assert lib.fft3d_stream_copy(4096, 8192, 15, None) == -1
    assert lib.fft3d_stream_copy(4104, 8192, 16, None) == -6
    assert lib.fft3d_stream_copy(4096, 8200, 16, None) == -6
    assert lib.fft3d_stream_copy(None, None, 0, None) == 0


def test_strerror_covers_codes():
    lib = _lib().lib()
    seen = set()
    for c in range(0, -10, -1):
        s = lib.fft3d_strerror(c).decode()
        assert s and s != "unknown status"
        seen.add(s)
    assert len(seen) == 10
    assert lib.fft3d_strerror(-99).decode() == "unknown status"


def test_no_device_reported_on_cpu_host():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    lib = _lib().lib()
    assert not lib.fft3d_plan(16, 16, 16, 1, 0, -1)
    assert lib.fft3d_last_error() == -3


def test_python_layer_raises_without_device():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    import paper_2006_08435_amd as fft3d
    with pytest.raises(fft3d.Fft3dError):
        fft3d.Plan(16, 16, 16)


def test_plan_many_rejects_bad_arguments():
    import ctypes
    L = _lib()
    lib = L.lib()

    def call(ns, bs, prec=0, direction=-1, count=None):
        k = len(ns)
        a = (ctypes.c_int * max(k, 1))(*ns)
        b = (ctypes.c_int * max(k, 1))(*bs)
        p = lib.fft3d_plan_many(k if count is None else count, ctypes.cast(a, ctypes.c_void_p),
                                ctypes.cast(a, ctypes.c_void_p), ctypes.cast(a, ctypes.c_void_p),
                                ctypes.cast(b, ctypes.c_void_p), prec, direction)
        assert not p
        return lib.fft3d_last_error()

    assert call([64], [1], count=0) == L.FFT3D_E_INVALID_ARG
    assert call([64] * 17, [1] * 17) == L.FFT3D_E_INVALID_ARG
    assert call([64], [0]) == L.FFT3D_E_INVALID_ARG
    assert call([64], [1], prec=5) == L.FFT3D_E_INVALID_ARG
    assert call([64], [1], direction=0) == L.FFT3D_E_INVALID_ARG
    assert call([7], [1]) == L.FFT3D_E_UNSUPPORTED_SIZE
    assert call([16], [1]) == L.FFT3D_E_UNSUPPORTED       # not a persistent-kernel size
    assert call([64], [1], prec=1) == L.FFT3D_E_UNSUPPORTED
    assert lib.fft3d_exec_many(None, None, None, None) == L.FFT3D_E_INVALID_ARG
    assert lib.fft3d_plan_set_schedule(None, 1024, 2) == L.FFT3D_E_INVALID_ARG
