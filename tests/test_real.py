"""Real-grid transforms (fft3d_plan_real: r2c forward, c2r inverse) on the GPU.

Densities and potentials are real (Section I's plane-wave operators), so
their transform under Eq. (1) is kept as the kx <= Nx/2 half.  Bars: the FP32
tolerance (relative L2 <= 5e-6) against the FP64 oracle's r2c3d / c2r3d on the
same float32 / complex64 inputs; the c2r is checked on arbitrary (not
Hermitian) half spectra, so the handling of the kx = 0 and Nx/2 entries is
pinned too.
"""
import numpy as np
import pytest

import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 5e-6
INVERSE, FORWARD = 1, -1
EVEN = [2, 4, 6, 8, 10, 12, 16, 18, 20, 24, 30, 32, 36, 40, 48, 50, 54, 60, 64, 72, 80, 90, 96, 100, 108,
        120, 128]


@pytest.fixture(scope="module")
def fft3d():
    import paper_2006_08435_amd as m
    assert torch.cuda.is_available()
    return m


def rel(a, b):
    a = np.asarray(a, np.complex128).ravel()
    b = np.asarray(b, np.complex128).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def real_input(n, nz, b, seed):
    return np.random.default_rng(seed).uniform(-1, 1, (b, nz, n, n)).astype(np.float32)


def half_input(n, nz, b, seed):
    rng = np.random.default_rng(seed)
    h = rng.uniform(-1, 1, (b, nz, n, n // 2 + 1)) + 1j * rng.uniform(-1, 1, (b, nz, n, n // 2 + 1))
    return h.astype(np.complex64)


def run(fft3d, x, direction, n):
    b, nz = x.shape[0], x.shape[1]
    plan = fft3d.RealPlan(n, n, nz, b, direction)
    xt = torch.from_numpy(np.ascontiguousarray(x)).cuda()
    y = plan.exec(xt)
    torch.cuda.synchronize()
    return y.cpu().numpy(), plan


@pytest.mark.parametrize("n", EVEN)
def test_r2c_all_even_sizes(fft3d, n):
    b = 3 if n <= 32 else 1
    f = real_input(n, n, b, 9000 + n)
    got, plan = run(fft3d, f, FORWARD, n)
    assert got.shape == (b, n, n, n // 2 + 1)
    want = oracle.r2c3d(f.astype(np.float64))
    for j in range(b):
        assert rel(got[j], want[j]) <= TOL, (n, j)


@pytest.mark.parametrize("n", EVEN)
def test_c2r_all_even_sizes(fft3d, n):
    b = 3 if n <= 32 else 1
    h = half_input(n, n, b, 9100 + n)
    got, plan = run(fft3d, h, INVERSE, n)
    assert got.shape == (b, n, n, n)
    want = oracle.c2r3d(h.astype(np.complex128), n)
    for j in range(b):
        assert rel(got[j], want[j]) <= TOL, (n, j)


@pytest.mark.parametrize("n,nz,b", [(48, 30, 2), (24, 5, 3), (16, 1, 2), (64, 27, 1), (10, 128, 1)])
def test_noncubic_depth(fft3d, n, nz, b):
    f = real_input(n, nz, b, 9200 + n + nz)
    got, _ = run(fft3d, f, FORWARD, n)
    assert rel(got, oracle.r2c3d(f.astype(np.float64))) <= TOL
    h = half_input(n, nz, b, 9300 + n + nz)
    got, _ = run(fft3d, h, INVERSE, n)
    assert rel(got, oracle.c2r3d(h.astype(np.complex128), n)) <= TOL


@pytest.mark.parametrize("n", [32, 96, 128])
def test_round_trip(fft3d, n):
    f = real_input(n, n, 2, 9400 + n)
    fwd = fft3d.RealPlan(n, n, n, 2, FORWARD)
    inv = fft3d.RealPlan(n, n, n, 2, INVERSE)
    ft = torch.from_numpy(f).cuda()
    back = inv.exec(fwd.exec(ft))
    torch.cuda.synchronize()
    assert rel(back.cpu().numpy() / n ** 3, f) <= TOL


def test_full_size_batch(fft3d):
    """32 real grids of 128^3, sampled grids against the oracle."""
    n, b = 128, 32
    f = real_input(n, n, b, 9500)
    got, _ = run(fft3d, f, FORWARD, n)
    for j in (0, 17, b - 1):
        assert rel(got[j], oracle.r2c3d(f[j].astype(np.float64))) <= TOL, j


def test_passes_compose(fft3d):
    n = 64
    lib = fft3d._lib.lib()
    s = torch.cuda.current_stream().cuda_stream
    for direction in (FORWARD, INVERSE):
        plan = fft3d.RealPlan(n, n, n, 2, direction)
        assert lib.fft3d_plan_passes(plan.handle) == 2
        if direction == FORWARD:
            x = torch.from_numpy(real_input(n, n, 2, 9600)).cuda()
            ref = plan.exec(x)
            out = torch.empty_like(ref)
            assert lib.fft3d_exec_pass(plan.handle, 0, x.data_ptr(), out.data_ptr(), s) == 0
            # the z pass works in place on `out` whatever `in` is (here the
            # smaller real buffer, which it must not read)
            assert lib.fft3d_exec_pass(plan.handle, 1, x.data_ptr(), out.data_ptr(), s) == 0
        else:
            h = torch.from_numpy(half_input(n, n, 2, 9700)).cuda()
            h2 = h.clone()
            ref = plan.exec(h)
            out = torch.empty_like(ref)
            assert lib.fft3d_exec_pass(plan.handle, 0, h2.data_ptr(), out.data_ptr(), s) == 0
            assert lib.fft3d_exec_pass(plan.handle, 1, h2.data_ptr(), out.data_ptr(), s) == 0
        torch.cuda.synchronize()
        assert torch.equal(ref, out)


def test_rejections(fft3d):
    lib = fft3d._lib.lib()
    for args in ((15, 15, 15, 1, -1), (32, 16, 32, 1, -1), (9, 9, 4, 1, 1)):
        assert not lib.fft3d_plan_real(*args)
        assert lib.fft3d_last_error() == -7
    assert not lib.fft3d_plan_real(14, 14, 14, 1, -1)
    assert lib.fft3d_last_error() == -2
    p = fft3d.RealPlan(32, 32, 32, 1, FORWARD)
    assert lib.fft3d_real_bytes(p.handle) == 32 ** 3 * 4
    x = torch.zeros(32 ** 3 * 4, dtype=torch.float32, device="cuda")
    s = torch.cuda.current_stream().cuda_stream
    assert lib.fft3d_exec(p.handle, x.data_ptr(), x.data_ptr(), s) == -1
    assert lib.fft3d_plan_set_cutoff(p.handle, 10.0) == -7
    q = fft3d.Plan(32, 32, 32, 1, "fp32", INVERSE)
    assert lib.fft3d_real_bytes(q.handle) == 0
