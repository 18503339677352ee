"""Differentiable transforms and the plane-wave local-potential energy.

* FFT3D / IFFT3D: the unnormalised forward (Eq. (1), sign -1) and inverse
  (sign +1) transforms as autograd functions; the backward of each is the
  other one, since the adjoint (conjugate transpose) of the unnormalised
  forward DFT is the unnormalised inverse.
* LocalPotentialEnergy: E = sum_n sum_r V(r) |psi_n(r)|^2 with
  psi_n = IFFT3D(c_n), computed by fft3d_energy_fwd (inverse transform with
  the sum fused into its last pass); backward = fft3d_energy_bwd, i.e.
  grad_c = FFT3D(2 gE V psi), with the 2 gE V factor fused into the first
  pass.  With save_psi=False the forward is fft3d_energy (E only, psi never
  written) and the backward recomputes psi inside the fused operator.  Gradients follow PyTorch's convention for real functions of complex
  tensors: dE/dRe(c) + i dE/dIm(c).
"""
from __future__ import annotations

import torch

from . import _lib
from . import FFT3D_FORWARD, FFT3D_INVERSE, fftn, get_plan, ifftn


class FFT3D(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x):
        return fftn(x)

    @staticmethod
    def backward(ctx, g):
        return ifftn(g.contiguous())


class IFFT3D(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x):
        return ifftn(x)

    @staticmethod
    def backward(ctx, g):
        return fftn(g.contiguous())


def _check_energy_args(c, V):
    if c.dtype != torch.complex64 or not c.is_cuda:
        raise TypeError("c must be a complex64 device tensor")
    if V.dtype != torch.float32 or not V.is_cuda or V.dim() != 3:
        raise TypeError("V must be a float32 device tensor [Nz, Ny, Nx]")
    cb = c.unsqueeze(0) if c.dim() == 3 else c
    if cb.dim() != 4 or tuple(cb.shape[1:]) != tuple(V.shape):
        raise ValueError("c %s and V %s shapes differ" % (tuple(c.shape), tuple(V.shape)))
    return cb.contiguous(), V.contiguous()


class LocalPotentialEnergy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, c, V, save_psi=True):
        cb, Vc = _check_energy_args(c, V)
        b, nz, ny, nx = cb.shape
        plan = get_plan(nx, ny, nz, b, "fp32", FFT3D_INVERSE)
        psi = torch.empty_like(cb)   # psi, or the intermediate of the E-only pass
        E = torch.empty((), dtype=torch.float64, device=cb.device)
        sh = int(torch.cuda.current_stream().cuda_stream)
        if save_psi:
            _lib.check(_lib.lib().fft3d_energy_fwd(plan.handle, cb.data_ptr(), Vc.data_ptr(), psi.data_ptr(),
                                                   E.data_ptr(), sh), "fft3d_energy_fwd")
        else:   # psi is recomputed by the backward: E alone, psi never written
            _lib.check(_lib.lib().fft3d_energy(plan.handle, cb.data_ptr(), Vc.data_ptr(), psi.data_ptr(),
                                               E.data_ptr(), sh), "fft3d_energy")
        ctx.save_for_backward(psi if save_psi else cb, Vc)
        ctx.have_psi = bool(save_psi)
        ctx.squeeze = c.dim() == 3
        ctx.plan = plan
        return E

    @staticmethod
    def backward(ctx, gE):
        src, Vc = ctx.saved_tensors
        grad = torch.empty_like(src)
        g64 = gE.detach().to(torch.float64).reshape(()).contiguous()
        sh = int(torch.cuda.current_stream().cuda_stream)
        _lib.check(_lib.lib().fft3d_energy_bwd(ctx.plan.handle, src.data_ptr(), int(ctx.have_psi), Vc.data_ptr(),
                                               g64.data_ptr(), grad.data_ptr(), sh), "fft3d_energy_bwd")
        if ctx.squeeze:
            grad = grad[0]
        return grad, None, None


def local_potential_energy(c, V, save_psi: bool = True):
    """E = sum_n sum_r V(r) |IFFT3D(c_n)(r)|^2 (differentiable in c)."""
    return LocalPotentialEnergy.apply(c, V, save_psi)


def energy(c, V):
    """E alone (fft3d_energy: psi is summed on chip and never written)."""
    cb, Vc = _check_energy_args(c, V)
    b, nz, ny, nx = cb.shape
    plan = get_plan(nx, ny, nz, b, "fp32", FFT3D_INVERSE)
    work = torch.empty_like(cb)
    E = torch.empty((), dtype=torch.float64, device=cb.device)
    sh = int(torch.cuda.current_stream().cuda_stream)
    _lib.check(_lib.lib().fft3d_energy(plan.handle, cb.data_ptr(), Vc.data_ptr(), work.data_ptr(), E.data_ptr(), sh),
               "fft3d_energy")
    return E


def energy_and_psi(c, V):
    """(E, psi) without autograd: one fused inverse pass."""
    cb, Vc = _check_energy_args(c, V)
    b, nz, ny, nx = cb.shape
    plan = get_plan(nx, ny, nz, b, "fp32", FFT3D_INVERSE)
    psi = torch.empty_like(cb)
    E = torch.empty((), dtype=torch.float64, device=cb.device)
    sh = int(torch.cuda.current_stream().cuda_stream)
    _lib.check(_lib.lib().fft3d_energy_fwd(plan.handle, cb.data_ptr(), Vc.data_ptr(), psi.data_ptr(),
                                           E.data_ptr(), sh), "fft3d_energy_fwd")
    return E, (psi[0] if c.dim() == 3 else psi)
