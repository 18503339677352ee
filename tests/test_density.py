"""Electron density rho = sum_n f_n |inverse(c_n)|^2 on the GPU
(fft3d_density: inverse xy planes, then one kernel per group of z-lines that
transforms every orbital in turn and sums f |psi|^2 in registers), against
the FP64 oracle's density.  Bar: relative L2 <= 5e-6 (FP32 tolerance; rho is
a sum of non-negative terms, so no cancellation)."""
import numpy as np
import pytest

import oracle
import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 5e-6


@pytest.fixture(scope="module")
def F():
    import paper_2006_08435_amd as m
    assert torch.cuda.is_available()
    return m


def rel(a, b):
    a = np.asarray(a, np.float64).ravel()
    b = np.asarray(b, np.float64).ravel()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def orbitals(shape, b, seed):
    c = np.stack([workloads.sphere_grid(shape, seed + j) for j in range(b)])
    occ = np.random.default_rng(seed).uniform(0.0, 2.0, b).astype(np.float32)
    return c, occ


@pytest.mark.parametrize("shape,b", [((16, 16, 16), 3), ((32, 32, 32), 4), ((48, 48, 30), 2), ((64, 64, 64), 2),
                                     ((96, 96, 96), 2), ((128, 128, 128), 1), ((25, 25, 27), 3), ((60, 60, 1), 2)])
def test_density_matches_oracle(F, shape, b):
    nx, ny, nz = shape
    c, occ = orbitals(shape, b, 13000 + nx + nz)
    plan = F.Plan(nx, ny, nz, b, "fp32", 1)
    rho = plan.density(torch.from_numpy(c).cuda(), torch.from_numpy(occ).cuda())
    torch.cuda.synchronize()
    want = oracle.density(c.astype(np.complex128), occ.astype(np.float64))
    assert rel(rho.cpu().numpy(), want) <= TOL


def test_in_place_and_deterministic(F):
    shape, b = (64, 64, 64), 5
    c, occ = orbitals(shape, b, 13100)
    plan = F.Plan(64, 64, 64, b, "fp32", -1)
    ct = torch.from_numpy(c).cuda()
    ot = torch.from_numpy(occ).cuda()
    r1 = plan.density(ct, ot)
    r2 = plan.density(ct, ot)
    work = ct.clone()
    r3 = plan.density(work, ot, work=work)         # work == c: c is overwritten
    torch.cuda.synchronize()
    assert torch.equal(r1, r2) and torch.equal(r1, r3)


@pytest.mark.parametrize("n,b,r2", [(32, 3, 64.0), (96, 2, 576.0), (128, 2, 1024.0)])
def test_density_with_cutoff(F, n, b, r2):
    c, occ = orbitals(n, b, 13200 + n)
    g = workloads.signed_freq(n)
    m = (g[:, None, None] ** 2 + g[None, :, None] ** 2 + g[None, None, :] ** 2) < r2
    c = (c * m[None]).astype(np.complex64)
    plan = F.Plan(n, n, n, b, "fp32", 1)
    plan.set_cutoff(r2)
    rho = plan.density(torch.from_numpy(c).cuda(), torch.from_numpy(occ).cuda())
    torch.cuda.synchronize()
    assert rel(rho.cpu().numpy(), oracle.density(c.astype(np.complex128), occ.astype(np.float64))) <= TOL


def test_orbital_batch_96(F):
    """32 orbitals at 96^3 (sphere-cutoff coefficients), rho over all of them."""
    n, B = 96, 32
    c = np.stack([workloads.sphere_grid(n, workloads.SEED_ORBITALS + j) for j in range(B)])
    occ = np.full(B, 2.0, np.float32)
    plan = F.Plan(n, n, n, B, "fp32", 1)
    rho = plan.density(torch.from_numpy(c).cuda(), torch.from_numpy(occ).cuda())
    torch.cuda.synchronize()
    assert rel(rho.cpu().numpy(), oracle.density(c.astype(np.complex128), occ.astype(np.float64))) <= TOL


def test_rejections(F):
    lib = F._lib.lib()
    s = torch.cuda.current_stream().cuda_stream
    x = torch.zeros((1, 16, 16, 24), dtype=torch.complex64, device="cuda")
    occ = torch.ones(1, dtype=torch.float32, device="cuda")
    rho = torch.zeros((16, 16, 24), dtype=torch.float32, device="cuda")
    p = F.Plan(24, 16, 16, 1, "fp32", 1)               # nx != ny
    assert lib.fft3d_density(p.handle, x.data_ptr(), occ.data_ptr(), rho.data_ptr(), x.data_ptr(), s) == -7
    q = F.Plan(24, 24, 16, 1, "fp32", 1)
    assert lib.fft3d_density(q.handle, x.data_ptr() + 8, occ.data_ptr(), rho.data_ptr(), x.data_ptr(), s) == -6
