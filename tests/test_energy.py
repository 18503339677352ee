"""Differentiation form: E = sum V |IFFT(c)|^2 and its gradient on the GPU,
against the FP64 oracle, exact central differences and the adjoint identity."""
import numpy as np
import pytest

import oracle
import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


# FP32 transforms and gradients are held to relative L2 error 5e-6 against
# FP64; the scalar E = sum V|psi|^2 to relative error 1e-6 (its FP32 products
# are summed in FP64; measured 1.9e-7 on the 128 x 96^3 orbital batch).
E_TOL = 1e-6


def rel(a, b):
    a = np.asarray(a, np.complex128).ravel()
    b = np.asarray(b, np.complex128).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(scope="module")
def F():
    import paper_2006_08435_amd as m
    from paper_2006_08435_amd import autograd  # noqa: F401
    return m


def make(shape, b, seed):
    nx, ny, nz = shape
    c = np.stack([workloads.sphere_grid(shape, seed + j) for j in range(b)])
    V = workloads.smooth_potential(shape, seed + 999)
    return c, V


@pytest.mark.parametrize("shape,b", [((16, 16, 16), 3), ((24, 24, 20), 2), ((64, 64, 64), 2), ((96, 96, 96), 2),
                                     ((128, 128, 32), 1), ((30, 30, 30), 4)])
def test_energy_and_gradient_match_oracle(F, shape, b):
    c, V = make(shape, b, 7000 + sum(shape))
    E_ref, psi_ref, g_ref = oracle.energy(c.astype(np.complex128), V.astype(np.float64), want_psi=True)
    ct = torch.from_numpy(c).cuda().requires_grad_(True)
    Vt = torch.from_numpy(V).cuda()
    E = F.local_potential_energy(ct, Vt)
    E.backward()
    torch.cuda.synchronize()
    assert abs(E.item() - E_ref) <= E_TOL * abs(E_ref), (E.item(), E_ref)
    assert rel(ct.grad.cpu().numpy(), g_ref) <= 5e-6
    E2, psi = F.energy_and_psi(ct.detach(), Vt)
    assert rel(psi.cpu().numpy(), psi_ref) <= 5e-6
    assert E2.item() == E.item()            # same fused reduction, fixed order


@pytest.mark.parametrize("shape,b", [((16, 16, 16), 3), ((24, 24, 20), 2), ((96, 96, 96), 2), ((30, 30, 30), 4),
                                     ((8, 8, 1), 2), ((128, 128, 16), 1)])
def test_energy_only_equals_fused_forward(F, shape, b):
    """fft3d_energy sums the same FP32 products in the same FP64 order as
    fft3d_energy_fwd (bit-identical E) and leaves c intact; with work == c it
    overwrites c and gives the same E."""
    c, V = make(shape, b, 7300 + sum(shape))
    ct = torch.from_numpy(c).cuda()
    Vt = torch.from_numpy(V).cuda()
    E_fwd, _ = F.energy_and_psi(ct, Vt)
    E_only = F.energy(ct, Vt)
    torch.cuda.synchronize()
    assert E_only.item() == E_fwd.item()
    assert torch.equal(ct.cpu(), torch.from_numpy(c))
    E_ref, _, _ = oracle.energy(c.astype(np.complex128), V.astype(np.float64), want_grad=False)
    assert abs(E_only.item() - E_ref) <= E_TOL * abs(E_ref)
    lib = F._lib.lib()
    E2 = torch.zeros((), dtype=torch.float64, device="cuda")
    plan = F.get_plan(shape[0], shape[1], shape[2], b, "fp32", F.FFT3D_INVERSE)
    sh = int(torch.cuda.current_stream().cuda_stream)
    assert lib.fft3d_energy(plan.handle, ct.data_ptr(), Vt.data_ptr(), ct.data_ptr(), E2.data_ptr(), sh) == 0
    torch.cuda.synchronize()
    assert E2.item() == E_fwd.item()


def test_energy_only_rejections(F):
    lib = F._lib.lib()
    c = torch.zeros((1, 16, 16, 16), dtype=torch.complex64, device="cuda")
    V = torch.zeros((16, 16, 16), dtype=torch.float32, device="cuda")
    E = torch.zeros((), dtype=torch.float64, device="cuda")
    p = F.Plan(16, 16, 16, 1, "fp32", F.FFT3D_INVERSE)
    assert lib.fft3d_energy(p.handle, c.data_ptr(), V.data_ptr(), None, E.data_ptr(), None) == -1
    assert lib.fft3d_energy(p.handle, c.data_ptr() + 8, V.data_ptr(), c.data_ptr(), E.data_ptr(), None) == -6
    q = F.Plan(16, 16, 16, 1, "fp16", F.FFT3D_INVERSE)
    assert lib.fft3d_energy(q.handle, c.data_ptr(), V.data_ptr(), c.data_ptr(), E.data_ptr(), None) == -7


def test_saved_psi_and_recompute_agree(F):
    c, V = make((48, 48, 48), 3, 123)
    Vt = torch.from_numpy(V).cuda()
    grads = []
    for save in (True, False):
        ct = torch.from_numpy(c).cuda().requires_grad_(True)
        F.local_potential_energy(ct, Vt, save).backward()
        grads.append(ct.grad.clone())
    torch.cuda.synchronize()
    assert rel(grads[0].cpu().numpy(), grads[1].cpu().numpy()) <= 1e-6


def test_upstream_gradient_scales(F):
    c, V = make((32, 32, 32), 2, 55)
    Vt = torch.from_numpy(V).cuda()
    ct = torch.from_numpy(c).cuda().requires_grad_(True)
    (3.5 * F.local_potential_energy(ct, Vt)).backward()
    g1 = ct.grad.clone()
    ct.grad = None
    F.local_potential_energy(ct, Vt).backward()
    assert rel((g1 / 3.5).cpu().numpy(), ct.grad.cpu().numpy()) <= 1e-6


def test_central_difference_is_exact(F):
    """E is quadratic in c, so (E(c+ed) - E(c-ed)) / 2e = Re<grad, d> exactly;
    a step with e|d| ~ |c| keeps FP32 rounding far below the signal."""
    c, V = make((64, 64, 64), 2, 77)
    Vt = torch.from_numpy(V).cuda()
    ct = torch.from_numpy(c).cuda().requires_grad_(True)
    F.local_potential_energy(ct, Vt).backward()
    g = ct.grad.cpu().numpy().astype(np.complex128)
    rng = np.random.default_rng(5)
    d = (rng.standard_normal(c.shape) + 1j * rng.standard_normal(c.shape)) * (np.abs(c) > 0)
    eps = np.linalg.norm(c) / np.linalg.norm(d)
    with torch.no_grad():
        Ep = F.local_potential_energy(torch.from_numpy((c + eps * d).astype(np.complex64)).cuda(), Vt).item()
        Em = F.local_potential_energy(torch.from_numpy((c - eps * d).astype(np.complex64)).cuda(), Vt).item()
    fd = (Ep - Em) / (2 * eps)
    lin = float(np.real(np.vdot(g, d.astype(np.complex64).astype(np.complex128))))
    assert abs(fd - lin) <= 1e-5 * (abs(Ep) + abs(Em)) / eps


def test_adjoint_dot_identity(F):
    """<F x, y> = <x, F^H y> with F^H the unnormalised inverse."""
    n = 48
    x = workloads.uniform_grid(n, 1, batch=2)
    y = workloads.uniform_grid(n, 2, batch=2)
    Fx = F.fftn(torch.from_numpy(x).cuda()).cpu().numpy().astype(np.complex128)
    FHy = F.ifftn(torch.from_numpy(y).cuda()).cpu().numpy().astype(np.complex128)
    lhs = np.vdot(y.astype(np.complex128), Fx)
    rhs = np.vdot(FHy, x.astype(np.complex128))
    assert abs(lhs - rhs) <= 1e-5 * abs(lhs)


def test_fft_autograd_matches_oracle(F):
    """L = sum w |FFT3D(x)|^2 -> grad = 2 IFFT(w FFT(x)) (oracle)."""
    n = 32
    x = workloads.uniform_grid(n, 3, batch=2)
    w = workloads.smooth_potential(n, 4)
    xt = torch.from_numpy(x).cuda().requires_grad_(True)
    y = F.FFT3D.apply(xt)
    L = (torch.from_numpy(w).cuda() * (y.real ** 2 + y.imag ** 2)).sum()
    L.backward()
    Y = oracle.fft3d(x.astype(np.complex128), -1)
    ref = 2 * oracle.fft3d(w * Y, 1)
    assert rel(xt.grad.cpu().numpy(), ref) <= 5e-6
    xt.grad = None
    z = F.IFFT3D.apply(xt)
    L = (torch.from_numpy(w).cuda() * (z.real ** 2 + z.imag ** 2)).sum()
    L.backward()
    Z = oracle.fft3d(x.astype(np.complex128), 1)
    ref = 2 * oracle.fft3d(w * Z, -1)
    assert rel(xt.grad.cpu().numpy(), ref) <= 5e-6


def test_energy_deterministic(F):
    c, V = make((64, 64, 64), 4, 99)
    ct = torch.from_numpy(c).cuda()
    Vt = torch.from_numpy(V).cuda()
    vals = [F.energy_and_psi(ct, Vt)[0].item() for _ in range(5)]
    assert len(set(vals)) == 1


def test_energy_rejects_unsupported(F):
    from paper_2006_08435_amd import _lib
    p = F.Plan(16, 8, 8, 1, "fp32", 1)
    t = torch.zeros(16 * 8 * 8, dtype=torch.complex64, device="cuda")
    V = torch.zeros(16 * 8 * 8, dtype=torch.float32, device="cuda")
    E = torch.zeros(1, dtype=torch.float64, device="cuda")
    assert _lib.lib().fft3d_energy_fwd(p.handle, t.data_ptr(), V.data_ptr(), t.data_ptr(), E.data_ptr(),
                                       None) == _lib.FFT3D_E_UNSUPPORTED
    assert _lib.lib().fft3d_energy_fwd(p.handle, None, V.data_ptr(), t.data_ptr(), E.data_ptr(),
                                       None) == _lib.FFT3D_E_INVALID_ARG


def test_orbital_batch_128x96(F):
    """128 orbitals at 96^3 (the large differentiation workload)."""
    B, n = 128, 96
    c = np.stack([workloads.sphere_grid(n, workloads.SEED_ORBITALS + j) for j in range(B)])
    V = workloads.smooth_potential(n, workloads.SEED_POTENTIAL)
    ct = torch.from_numpy(c).cuda().requires_grad_(True)
    Vt = torch.from_numpy(V).cuda()
    E = F.local_potential_energy(ct, Vt, save_psi=False)   # E alone, psi recomputed in backward
    E.backward()
    E_psi, _ = F.energy_and_psi(ct.detach(), Vt)             # E with psi stored
    torch.cuda.synchronize()
    assert E_psi.item() == E.item()
    E_ref, _, g_ref = oracle.energy(c.astype(np.complex128), V.astype(np.float64))
    assert abs(E.item() - E_ref) <= E_TOL * abs(E_ref), (E.item(), E_ref)
    assert rel(ct.grad.cpu().numpy(), g_ref) <= 5e-6
