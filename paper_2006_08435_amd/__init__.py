"""MI355X-native complex 3D FFT (the hot path of Ramaswami et al., Section II).

Thin Python layer over the C ABI in ``include/fft3d.h`` (``libfft3d.so``):
PyTorch supplies device memory and the current HIP stream; every step of the
transform runs in the library's HIP kernels.

    import paper_2006_08435_amd as fft3d
    y = fft3d.fftn(x)        # x: complex64 CUDA tensor [B, Nz, Ny, Nx] or [Nz, Ny, Nx]
    z = fft3d.ifftn(y)       # unnormalised: z == Nx*Ny*Nz * x
"""
from __future__ import annotations

import threading

from . import _lib
from ._lib import (FFT3D_BF16_SCALED, FFT3D_FORWARD, FFT3D_FP16_SCALED, FFT3D_FP32,
                   FFT3D_INVERSE, Fft3dError)

PRECISIONS = {"fp32": FFT3D_FP32, "fp16": FFT3D_FP16_SCALED, "bf16": FFT3D_BF16_SCALED}


def _torch():
    import torch
    return torch


def _stream_handle(stream=None) -> int:
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


class Plan:
    """A planned batch of nx*ny*nz transforms (owns its device tables)."""

    def __init__(self, nx: int, ny: int, nz: int, batch: int = 1, precision="fp32",
                 direction: int = FFT3D_FORWARD):
        lib = _lib.lib()
        prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        h = lib.fft3d_plan(int(nx), int(ny), int(nz), int(batch), prec, int(direction))
        if not h:
            raise Fft3dError(lib.fft3d_last_error(), "fft3d_plan(%d,%d,%d,%d)" % (nx, ny, nz, batch))
        self._h = h
        self.shape = (int(batch), int(nz), int(ny), int(nx))
        self.precision = prec
        self.direction = int(direction)

    @property
    def handle(self) -> int:
        return self._h

    @property
    def buffer_bytes(self) -> int:
        return int(_lib.lib().fft3d_buffer_bytes(self._h))

    def describe(self) -> str:
        import ctypes
        buf = ctypes.create_string_buffer(512)
        _lib.lib().fft3d_plan_describe(self._h, buf, 512)
        return buf.value.decode()

    def set_cutoff(self, r2: float) -> None:
        """Promise that the input vanishes wherever Gx^2+Gy^2+Gz^2 >= r2
        (signed frequencies) and prune the inverse accordingly; r2 <= 0
        restores the dense schedule (``fft3d_plan_set_cutoff``)."""
        _lib.check(_lib.lib().fft3d_plan_set_cutoff(self._h, float(r2)), "fft3d_plan_set_cutoff")

    @property
    def sphere_points(self) -> int:
        """Points per grid inside the cutoff sphere (a cutoff must be set)."""
        n = int(_lib.lib().fft3d_plan_sphere_points(self._h))
        _lib.check(min(n, 0), "fft3d_plan_sphere_points")
        return n

    def _packed_like(self, dense):
        torch = _torch()
        return torch.empty((self.shape[0], self.sphere_points), dtype=dense.dtype, device=dense.device)

    def _check_pair(self, dense, packed):
        for t in (dense, packed):
            if not t.is_cuda or not t.is_contiguous():
                raise ValueError("tensors must be contiguous device tensors")
        if dense.numel() * dense.element_size() != self.buffer_bytes:
            raise ValueError("dense tensor holds %d bytes, plan needs %d"
                             % (dense.numel() * dense.element_size(), self.buffer_bytes))
        if packed.numel() != self.shape[0] * self.sphere_points or packed.element_size() != 8:
            raise ValueError("packed tensor must hold batch * sphere_points complex64 values")

    def pack(self, dense, packed=None, stream=None):
        """Gather the points inside the cutoff sphere: [batch, sphere_points]."""
        if packed is None:
            packed = self._packed_like(dense)
        self._check_pair(dense, packed)
        _lib.check(_lib.lib().fft3d_sphere_pack(self._h, dense.data_ptr(), packed.data_ptr(),
                                                _stream_handle(stream)), "fft3d_sphere_pack")
        return packed

    def unpack(self, packed, dense=None, stream=None):
        """Scatter a packed sphere into a dense grid (zeros outside)."""
        torch = _torch()
        if dense is None:
            dense = torch.empty(self.shape, dtype=packed.dtype, device=packed.device)
        self._check_pair(dense, packed)
        _lib.check(_lib.lib().fft3d_sphere_unpack(self._h, packed.data_ptr(), dense.data_ptr(),
                                                  _stream_handle(stream)), "fft3d_sphere_unpack")
        return dense

    def exec_packed(self, dense, packed, stream=None):
        """Pruned transform with a packed sphere: inverse packed -> dense;
        forward dense -> packed (``dense`` is overwritten as workspace)."""
        self._check_pair(dense, packed)
        _lib.check(_lib.lib().fft3d_exec_packed(self._h, dense.data_ptr(), packed.data_ptr(),
                                                _stream_handle(stream)), "fft3d_exec_packed")
        return dense if self.direction == FFT3D_INVERSE else packed

    def apply_potential(self, c, V, out=None, E=None, scale=None, stream=None):
        """out = scale * forward(V * inverse(c)) (``fft3d_apply_potential``);
        E (a 0-d float64 device tensor) receives sum V |inverse(c)|^2."""
        torch = _torch()
        if out is None:
            out = torch.empty_like(c)
        for t in (c, out, V):
            if not t.is_cuda or not t.is_contiguous():
                raise ValueError("tensors must be contiguous device tensors")
        ptr = lambda t: 0 if t is None else t.data_ptr()
        _lib.check(_lib.lib().fft3d_apply_potential(self._h, c.data_ptr(), V.data_ptr(), out.data_ptr(), ptr(E),
                                                    ptr(scale), _stream_handle(stream)), "fft3d_apply_potential")
        return out

    def density(self, c, occ, rho=None, work=None, stream=None):
        """rho = sum_n occ[n] |inverse(c_n)|^2 (``fft3d_density``); work
        defaults to a fresh buffer (c is left intact)."""
        torch = _torch()
        if rho is None:
            rho = torch.empty(self.shape[1:], dtype=torch.float32, device=c.device)
        if work is None:
            work = torch.empty_like(c)
        for t in (c, occ, rho, work):
            if not t.is_cuda or not t.is_contiguous():
                raise ValueError("tensors must be contiguous device tensors")
        _lib.check(_lib.lib().fft3d_density(self._h, c.data_ptr(), occ.data_ptr(), rho.data_ptr(), work.data_ptr(),
                                            _stream_handle(stream)), "fft3d_density")
        return rho

    def exec_ptr(self, in_ptr: int, out_ptr: int, stream_handle: int) -> None:
        _lib.check(_lib.lib().fft3d_exec(self._h, in_ptr, out_ptr, stream_handle), "fft3d_exec")

    def exec(self, inp, out=None, stream=None):
        """Transform device tensor ``inp`` into ``out`` (allocated if None)."""
        torch = _torch()
        if out is None:
            out = torch.empty_like(inp)
        for t in (inp, out):
            if not t.is_cuda or not t.is_contiguous():
                raise ValueError("tensors must be contiguous device tensors")
            if t.numel() * t.element_size() != self.buffer_bytes:
                raise ValueError("tensor holds %d bytes, plan needs %d"
                                 % (t.numel() * t.element_size(), self.buffer_bytes))
        self.exec_ptr(inp.data_ptr(), out.data_ptr(), _stream_handle(stream))
        return out

    def close(self) -> None:
        if getattr(self, "_h", None):
            _lib.lib().fft3d_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class PlanMany:
    """Heterogeneous batch: groups of cubic grids transformed by one
    persistent launch.  ``groups`` is a list of (n, batch) pairs."""

    def __init__(self, groups, direction: int = FFT3D_FORWARD, precision="fp32"):
        import ctypes
        lib = _lib.lib()
        k = len(groups)
        arr = lambda vals: (ctypes.c_int * k)(*[int(v) for v in vals])
        ns = arr([g[0] for g in groups])
        bs = arr([g[1] for g in groups])
        prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        h = lib.fft3d_plan_many(k, ctypes.cast(ns, ctypes.c_void_p), ctypes.cast(ns, ctypes.c_void_p),
                                ctypes.cast(ns, ctypes.c_void_p), ctypes.cast(bs, ctypes.c_void_p), prec,
                                int(direction))
        if not h:
            raise Fft3dError(lib.fft3d_last_error(), "fft3d_plan_many(%r)" % (groups,))
        self._h = h
        self.groups = [(int(n), int(b)) for n, b in groups]
        self.direction = int(direction)

    @property
    def handle(self) -> int:
        return self._h

    def describe(self) -> str:
        import ctypes
        buf = ctypes.create_string_buffer(512)
        _lib.lib().fft3d_plan_describe(self._h, buf, 512)
        return buf.value.decode()

    def set_schedule(self, threads: int, chunk: int) -> None:
        _lib.check(_lib.lib().fft3d_plan_set_schedule(self._h, int(threads), int(chunk)), "set_schedule")

    def set_group_schedule(self, group: int, radix_order: int, z_lines: int) -> None:
        """Radix order (0 default, 1 alternative) and z-tile width (32 or
        64 lines) of group `group`'s plain passes."""
        _lib.check(_lib.lib().fft3d_plan_set_group_schedule(self._h, int(group), int(radix_order), int(z_lines)),
                   "set_group_schedule")

    def tune(self) -> None:
        _lib.check(_lib.lib().fft3d_plan_tune(self._h), "fft3d_plan_tune")

    def exec_ptrs(self, in_ptrs, out_ptrs, stream_handle: int) -> None:
        import ctypes
        k = len(self.groups)
        ia = (ctypes.c_void_p * k)(*in_ptrs)
        oa = (ctypes.c_void_p * k)(*out_ptrs)
        _lib.check(_lib.lib().fft3d_exec_many(self._h, ctypes.cast(ia, ctypes.c_void_p),
                                              ctypes.cast(oa, ctypes.c_void_p), stream_handle), "fft3d_exec_many")

    def exec(self, ins, outs=None, stream=None):
        torch = _torch()
        if outs is None:
            outs = [torch.empty_like(t) for t in ins]
        for (n, b), i, o in zip(self.groups, ins, outs):
            for t in (i, o):
                if not t.is_cuda or not t.is_contiguous() or t.numel() != b * n ** 3 or t.dtype != torch.complex64:
                    raise ValueError("group tensors must be contiguous complex64 [%d, %d, %d, %d]" % (b, n, n, n))
        self.exec_ptrs([t.data_ptr() for t in ins], [t.data_ptr() for t in outs], _stream_handle(stream))
        return outs

    def close(self) -> None:
        if getattr(self, "_h", None):
            _lib.lib().fft3d_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_cache = {}
_cache_lock = threading.Lock()


class RealPlan:
    """Real grids (nx == ny, nx even): r2c forward real [B,Nz,Ny,Nx] ->
    complex [B,Nz,Ny,Nx/2+1]; c2r inverse the reverse, unnormalised, with the
    complex input overwritten (``fft3d_plan_real``)."""

    def __init__(self, nx: int, ny: int, nz: int, batch: int = 1, direction: int = FFT3D_FORWARD):
        lib = _lib.lib()
        h = lib.fft3d_plan_real(int(nx), int(ny), int(nz), int(batch), int(direction))
        if not h:
            raise Fft3dError(lib.fft3d_last_error(), "fft3d_plan_real(%d,%d,%d,%d)" % (nx, ny, nz, batch))
        self._h = h
        self.real_shape = (int(batch), int(nz), int(ny), int(nx))
        self.half_shape = (int(batch), int(nz), int(ny), int(nx) // 2 + 1)
        self.direction = int(direction)

    @property
    def handle(self) -> int:
        return self._h

    def describe(self) -> str:
        import ctypes
        buf = ctypes.create_string_buffer(512)
        _lib.lib().fft3d_plan_describe(self._h, buf, 512)
        return buf.value.decode()

    def exec(self, inp, out=None, stream=None):
        torch = _torch()
        fwd = self.direction == FFT3D_FORWARD
        in_dtype, out_dtype = (torch.float32, torch.complex64) if fwd else (torch.complex64, torch.float32)
        in_shape, out_shape = (self.real_shape, self.half_shape) if fwd else (self.half_shape, self.real_shape)
        if out is None:
            out = torch.empty(out_shape, dtype=out_dtype, device=inp.device)
        for t, dt, sh in ((inp, in_dtype, in_shape), (out, out_dtype, out_shape)):
            if not t.is_cuda or not t.is_contiguous() or t.dtype != dt or tuple(t.shape) != sh:
                raise ValueError("expected a contiguous %s device tensor of shape %s" % (dt, sh))
        _lib.check(_lib.lib().fft3d_exec(self._h, inp.data_ptr(), out.data_ptr(), _stream_handle(stream)),
                   "fft3d_exec")
        return out

    def close(self) -> None:
        if getattr(self, "_h", None):
            _lib.lib().fft3d_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def rfftn(x):
    """Half spectrum (kx <= Nx/2) of real grids [B,Nz,Ny,Nx] or [Nz,Ny,Nx]."""
    xb, sq = _as_batch(x)
    b, nz, ny, nx = xb.shape
    y = RealPlan(nx, ny, nz, b, FFT3D_FORWARD).exec(xb.contiguous())
    return y[0] if sq else y


def irfftn(h, nx: int):
    """Unnormalised real inverse of half spectra [B,Nz,Ny,Nx/2+1] (the input
    is copied first, since the transform overwrites its input)."""
    hb, sq = _as_batch(h)
    b, nz, ny, _ = hb.shape
    y = RealPlan(nx, ny, nz, b, FFT3D_INVERSE).exec(hb.clone())
    return y[0] if sq else y


def get_plan(nx, ny, nz, batch=1, precision="fp32", direction=FFT3D_FORWARD) -> Plan:
    import torch
    key = (nx, ny, nz, batch, precision, direction, torch.cuda.current_device())
    with _cache_lock:
        p = _cache.get(key)
        if p is None:
            p = Plan(nx, ny, nz, batch, precision, direction)
            _cache[key] = p
        return p


def _as_batch(x):
    if x.dim() == 3:
        return x.unsqueeze(0), True
    if x.dim() == 4:
        return x, False
    raise ValueError("expected [Nz,Ny,Nx] or [B,Nz,Ny,Nx], got %s" % (tuple(x.shape),))


def _transform(x, direction, out=None):
    torch = _torch()
    if x.dtype != torch.complex64:
        raise TypeError("fp32 path takes complex64 tensors")
    xb, squeeze = _as_batch(x.contiguous())
    b, nz, ny, nx = xb.shape
    plan = get_plan(nx, ny, nz, b, "fp32", direction)
    o = torch.empty_like(xb) if out is None else out.view(xb.shape)
    plan.exec(xb, o)
    return o[0] if squeeze else o


def scaled16_bytes(shape) -> int:
    """Bytes of a scaled 16-bit buffer for complex data of `shape` (last axis = rows)."""
    n = 1
    for d in shape:
        n *= int(d)
    return 4 * n + n // int(shape[-1])


def quantize(x, precision="fp16", out=None, stream=None):
    """complex64 device tensor -> scaled 16-bit buffer (torch.uint8), rows = last axis."""
    torch = _torch()
    if x.dtype != torch.complex64 or not x.is_cuda:
        raise TypeError("quantize takes a complex64 device tensor")
    x = x.contiguous()
    C = int(x.shape[-1])
    rows = x.numel() // C
    if out is None:
        out = torch.empty(scaled16_bytes(x.shape), dtype=torch.uint8, device=x.device)
    _lib.check(_lib.lib().fft3d_quantize(PRECISIONS[precision], rows, C, x.data_ptr(), out.data_ptr(),
                                         _stream_handle(stream)), "fft3d_quantize")
    return out


def dequantize(buf, shape, precision="fp16", stream=None):
    """scaled 16-bit buffer -> complex64 device tensor of `shape` (exact values)."""
    torch = _torch()
    C = int(shape[-1])
    n = 1
    for d in shape:
        n *= int(d)
    out = torch.empty(tuple(int(d) for d in shape), dtype=torch.complex64, device=buf.device)
    _lib.check(_lib.lib().fft3d_dequantize(PRECISIONS[precision], n // C, C, buf.data_ptr(), out.data_ptr(),
                                           _stream_handle(stream)), "fft3d_dequantize")
    return out


def fftn(x, out=None):
    """Eq. (1) over the last three axes (sign -1, unnormalised)."""
    return _transform(x, FFT3D_FORWARD, out)


def ifftn(x, out=None):
    """Unnormalised inverse over the last three axes (sign +1)."""
    return _transform(x, FFT3D_INVERSE, out)


def __getattr__(name):
    # autograd wrappers are imported lazily (they need torch at import time)
    if name in ("FFT3D", "IFFT3D", "LocalPotentialEnergy", "local_potential_energy", "energy", "energy_and_psi"):
        from . import autograd
        return getattr(autograd, name)
    raise AttributeError(name)


def stream_copy(src, dst, stream=None):
    """Copy device tensor src into dst (same byte size, contiguous) with the
    library's streaming copy kernel: the measured HBM ceiling the transform
    passes are compared with."""
    nbytes = src.numel() * src.element_size()
    if not (src.is_contiguous() and dst.is_contiguous()) or dst.numel() * dst.element_size() != nbytes:
        raise ValueError("stream_copy takes two contiguous tensors of the same byte size")
    _lib.check(_lib.lib().fft3d_stream_copy(src.data_ptr(), dst.data_ptr(), nbytes, _stream_handle(stream)),
               "fft3d_stream_copy")
    return dst


__all__ = ["Plan", "PlanMany", "RealPlan", "rfftn", "irfftn", "get_plan", "quantize", "dequantize", "scaled16_bytes", "stream_copy", "fftn", "ifftn", "Fft3dError", "FFT3D_FORWARD",
           "FFT3D_INVERSE", "FFT3D_FP32", "FFT3D_FP16_SCALED", "FFT3D_BF16_SCALED"]
