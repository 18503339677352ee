"""GPU parity of the FP32 path against the FP64 oracle, through the C ABI.

Bar for the FP32 form: relative L2 error <= 5e-6 per
transform against the oracle on the very same complex64 inputs.
"""
import numpy as np
import pytest

import oracle
import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 5e-6


def smooth_sizes(limit=128):
    out = []
    for n in range(1, limit + 1):
        m = n
        for p in (2, 3, 5):
            while m % p == 0:
                m //= p
        if m == 1:
            out.append(n)
    return out


def rel(a, b):
    a = np.asarray(a, np.complex128).ravel()
    b = np.asarray(b, np.complex128).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(scope="module")
def fft3d():
    import paper_2006_08435_amd as m
    assert torch.cuda.is_available()
    return m


def run(fft3d, x, direction, inplace=False, stream=None):
    b, nz, ny, nx = x.shape
    plan = fft3d.get_plan(nx, ny, nz, b, "fp32", direction)
    xt = torch.from_numpy(np.ascontiguousarray(x)).cuda()
    if inplace:
        plan.exec(xt, xt, stream=stream)
        out = xt
    else:
        out = plan.exec(xt, stream=stream)
    torch.cuda.synchronize()
    return out.cpu().numpy(), xt.cpu().numpy()


@pytest.mark.parametrize("n", smooth_sizes(128))
@pytest.mark.parametrize("direction", [-1, 1])
def test_cubic_all_sizes(fft3d, n, direction):
    b = 3 if n <= 32 else 1
    x = workloads.uniform_grid(n, 10 * n + (direction > 0), batch=b)
    got, _ = run(fft3d, x, direction)
    ref = oracle.fft3d(x.astype(np.complex128), direction)
    for i in range(b):
        assert rel(got[i], ref[i]) <= TOL, (n, direction, i, rel(got[i], ref[i]))


NONCUBIC = [(2, 3, 5), (4, 6, 5), (8, 3, 10), (5, 1, 3), (1, 1, 1), (1, 7 - 2, 1), (16, 16, 1),
            (128, 16, 8), (30, 20, 12), (64, 64, 128), (120, 120, 48), (100, 128, 64), (1, 128, 1),
            (128, 1, 1), (1, 1, 128), (27, 25, 9), (48, 48, 5), (96, 96, 2)]


@pytest.mark.parametrize("shape", NONCUBIC)
@pytest.mark.parametrize("direction", [-1, 1])
def test_noncubic(fft3d, shape, direction):
    nx, ny, nz = shape
    b = 2
    x = workloads.uniform_grid(shape, nx * 7 + ny * 13 + nz, batch=b)
    got, _ = run(fft3d, x, direction)
    ref = oracle.fft3d(x.astype(np.complex128), direction)
    assert rel(got, ref) <= TOL, (shape, direction, rel(got, ref))


def test_small_uniform_vs_bruteforce(fft3d):
    """16^3 uniform input, seed 1001: GPU vs Eq. (1) summed term by term."""
    x = workloads.uniform_grid(16, workloads.SEED_SMALL_UNIFORM)[None]
    fwd, xin = run(fft3d, x, -1)
    assert np.array_equal(xin, x), "out-of-place call modified its input"
    ref = oracle.dft3d_naive(x.astype(np.complex128), -1)
    assert rel(fwd, ref) <= TOL
    back, _ = run(fft3d, fwd, 1)
    assert rel(back / 16 ** 3, x) <= TOL


@pytest.mark.parametrize("n", [64, 128])
def test_single_sphere_grid_forward_inverse(fft3d, n):
    x = workloads.sphere_grid(n, workloads.SEED_SINGLE[n])[None]
    for direction in (1, -1):
        got, _ = run(fft3d, x, direction)
        ref = oracle.fft3d(x.astype(np.complex128), direction)
        assert rel(got, ref) <= TOL, (n, direction, rel(got, ref))
    psi, _ = run(fft3d, x, 1)
    back, _ = run(fft3d, psi, -1)
    assert rel(back / n ** 3, x) <= TOL


@pytest.mark.parametrize("shape", [(16, 16, 16), (64, 64, 64), (48, 48, 48), (30, 20, 12), (128, 128, 8)])
def test_inplace_matches_out_of_place(fft3d, shape):
    nx, ny, nz = shape
    x = workloads.uniform_grid(shape, 99, batch=2)
    a, _ = run(fft3d, x, -1)
    b, _ = run(fft3d, x, -1, inplace=True)
    assert np.array_equal(a, b)


def test_deterministic_and_stream_ordered(fft3d):
    x = workloads.uniform_grid(64, 5, batch=4)
    a, _ = run(fft3d, x, -1)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        b, _ = run(fft3d, x, -1, stream=s)
    assert np.array_equal(a, b)


def test_invariants_on_gpu_output(fft3d):
    """Parseval and linearity hold on the GPU result (no oracle involved)."""
    n = 96
    f = workloads.uniform_grid(n, 1, batch=2)
    F, _ = run(fft3d, f, -1)
    e_f = np.vdot(f.astype(np.complex128), f.astype(np.complex128)).real
    e_F = np.vdot(F.astype(np.complex128), F.astype(np.complex128)).real
    assert abs(e_F - n ** 3 * e_f) <= 1e-5 * n ** 3 * e_f
    g = workloads.uniform_grid(n, 2, batch=2)
    G, _ = run(fft3d, g, -1)
    H, _ = run(fft3d, (f + (0.5 - 2j) * g).astype(np.complex64), -1)
    assert rel(H, F + (0.5 - 2j) * G) <= 1e-5


def test_full_batch_128(fft3d):
    """32 x 128^3 sphere-cutoff batch (the large FP32 workload): every grid
    against the oracle element by element, and by Parseval."""
    B, n = 32, 128
    x = np.empty((B, n, n, n), np.complex64)
    for j in range(B):
        x[j] = workloads.sphere_grid(n, workloads.SEED_BATCH128 + j)
    for direction in (1, -1):
        got, _ = run(fft3d, x, direction)
        for j in range(B):
            ref = oracle.fft3d(x[j].astype(np.complex128), direction)
            assert rel(got[j], ref) <= TOL, (direction, j, rel(got[j], ref))
        ef = np.sum(np.abs(x.astype(np.complex128)) ** 2, axis=(1, 2, 3))
        eF = np.sum(np.abs(got.astype(np.complex128)) ** 2, axis=(1, 2, 3))
        assert np.all(np.abs(eF - n ** 3 * ef) <= 1e-5 * n ** 3 * ef)


@pytest.mark.parametrize("n,batch", [(128, 2), (125, 3)])
@pytest.mark.parametrize("direction", [-1, 1])
def test_streaming_plane_pass(fft3d, n, batch, direction):
    """At n = 125 and 128 a plane pass of 32 MB or more uses streaming loads
    and stores, smaller ones the default policy.  Only the memory policy
    differs: the first grid of the larger batch equals the same grid
    transformed alone, and both meet the oracle."""
    x = workloads.uniform_grid(n, 4200 + n + (direction > 0), batch=batch)
    assert batch * n ** 3 * 8 >= 32 << 20 > n ** 3 * 8
    big, _ = run(fft3d, x, direction)
    one, _ = run(fft3d, x[:1], direction)
    assert np.array_equal(big[0], one[0])
    for j in (0, batch - 1):
        ref = oracle.fft3d(x[j].astype(np.complex128), direction)
        assert rel(big[j], ref) <= TOL, (j, rel(big[j], ref))


def test_exec_argument_errors(fft3d):
    from paper_2006_08435_amd import _lib
    lib = _lib.lib()
    p = fft3d.Plan(16, 16, 16, 1)
    t = torch.zeros(16 ** 3 + 2, dtype=torch.complex64, device="cuda")
    assert lib.fft3d_exec(p.handle, None, t.data_ptr(), None) == _lib.FFT3D_E_INVALID_ARG
    assert lib.fft3d_exec(p.handle, t.data_ptr() + 8, t.data_ptr(), None) == _lib.FFT3D_E_ALIGNMENT
    assert lib.fft3d_exec(p.handle, t.data_ptr(), t.data_ptr(), None) == _lib.FFT3D_OK
    torch.cuda.synchronize()


def test_injected_allocation_failure(fft3d, monkeypatch):
    from paper_2006_08435_amd import _lib
    monkeypatch.setenv("FFT3D_TEST_FAIL_ALLOC", "1")
    lib = _lib.lib()
    assert not lib.fft3d_plan(32, 32, 32, 1, 0, -1)
    assert lib.fft3d_last_error() == _lib.FFT3D_E_ALLOC
