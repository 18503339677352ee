"""fft3d_energy_noalloc through the C ABI: the energy E = sum V |IFFT(c)|^2
of fft3d_energy without a plan and without any allocation (its twiddle
tables and partial sums live in the library's fixed per-device array).

Bar: the same kernels, tables and summation order as fft3d_energy on a plan,
so E must equal that entry point's E bit for bit, and the FP64 oracle's E to
the energy tolerance (relative 1e-6); two calls in a row, the second smaller
(the array keeps the first call's contents), then graph replays."""
import numpy as np
import pytest

import oracle
import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

E_TOL = 1e-6


@pytest.fixture(scope="module")
def F():
    import paper_2006_08435_amd as m
    assert torch.cuda.is_available()
    return m


def inputs(shape, b, seed):
    c = np.stack([workloads.sphere_grid(shape, seed + j) for j in range(b)])
    V = workloads.smooth_potential(shape, seed + 999)
    return c, V


def energy_noalloc(L, shape, b, ct, Vt, work, E, stream):
    nx, ny, nz = shape
    return L.fft3d_energy_noalloc(nx, ny, nz, b, ct.data_ptr(), Vt.data_ptr(), work.data_ptr(), E.data_ptr(),
                                  int(stream.cuda_stream))


def energy_plan(F, L, shape, b, ct, Vt, stream):
    nx, ny, nz = shape
    plan = F.Plan(nx, ny, nz, b, "fp32", F.FFT3D_INVERSE)
    work = torch.empty_like(ct)
    E = torch.zeros((), dtype=torch.float64, device="cuda")
    assert L.fft3d_energy(plan.handle, ct.data_ptr(), Vt.data_ptr(), work.data_ptr(), E.data_ptr(),
                          int(stream.cuda_stream)) == 0
    torch.cuda.synchronize()
    return E.item()


def test_noalloc_equals_plan_energy_two_calls(F):
    """A large call, then a smaller one: each E equals fft3d_energy's bit for
    bit and the oracle's to 1e-6; c is left intact."""
    from paper_2006_08435_amd import _lib
    L = _lib.lib()
    stream = torch.cuda.current_stream()
    for shape, b, seed in (((96, 96, 96), 16, 8100), ((40, 40, 30), 3, 8200)):
        c, V = inputs(shape, b, seed)
        ct = torch.from_numpy(c).cuda()
        Vt = torch.from_numpy(V).cuda()
        work = torch.empty_like(ct)
        E = torch.full((), float("nan"), dtype=torch.float64, device="cuda")
        print("noalloc case", shape, b, flush=True)
        assert energy_noalloc(L, shape, b, ct, Vt, work, E, stream) == 0
        torch.cuda.synchronize()
        got = E.item()
        assert got == energy_plan(F, L, shape, b, ct, Vt, stream), shape
        assert torch.equal(ct.cpu(), torch.from_numpy(c))
        E_ref, _, _ = oracle.energy(c.astype(np.complex128), V.astype(np.float64), want_grad=False)
        assert abs(got - E_ref) <= E_TOL * abs(E_ref), (shape, got, E_ref)


def test_noalloc_in_place_and_graph_replays(F):
    """work == c (overwrites c), and the call captured in a HIP graph: every
    replay, with eager calls of other sizes between replays, gives the
    eager E."""
    from paper_2006_08435_amd import _lib
    L = _lib.lib()
    shape, b = (64, 64, 64), 4
    c, V = inputs(shape, b, 8300)
    Vt = torch.from_numpy(V).cuda()
    cur = torch.cuda.current_stream()
    ref = energy_plan(F, L, shape, b, torch.from_numpy(c).cuda(), Vt, cur)
    ct = torch.from_numpy(c).cuda()
    E = torch.zeros((), dtype=torch.float64, device="cuda")
    assert energy_noalloc(L, shape, b, ct, Vt, ct, E, cur) == 0   # in place: c is the work buffer
    torch.cuda.synchronize()
    assert E.item() == ref
    # capture (the array was looked up by the calls above)
    src = torch.from_numpy(c).cuda()
    work = torch.empty_like(src)
    s = torch.cuda.Stream()
    s.wait_stream(cur)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            assert energy_noalloc(L, shape, b, src, Vt, work, E, s) == 0
    cur.wait_stream(s)
    c2, V2 = inputs((30, 30, 20), 2, 8400)
    c2t, V2t = torch.from_numpy(c2).cuda(), torch.from_numpy(V2).cuda()
    E2 = torch.zeros((), dtype=torch.float64, device="cuda")
    for r in range(4):
        E.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert E.item() == ref, r
        # an eager call of another size overwrites the shared array between replays
        assert energy_noalloc(L, (30, 30, 20), 2, c2t, V2t, torch.empty_like(c2t), E2, cur) == 0
        torch.cuda.synchronize()


def test_noalloc_rejections(F):
    """Argument errors return before any launch."""
    from paper_2006_08435_amd import _lib
    L = _lib.lib()
    t = torch.zeros(16 * 16 * 16 + 2, dtype=torch.complex64, device="cuda")
    v = torch.zeros(16 * 16 * 16, dtype=torch.float32, device="cuda")
    e = torch.zeros(2, dtype=torch.float64, device="cuda")
    p, q, r = t.data_ptr(), v.data_ptr(), e.data_ptr()
    f = L.fft3d_energy_noalloc
    assert f(16, 16, 16, 1, None, q, p, r, None) == _lib.FFT3D_E_INVALID_ARG
    assert f(16, 16, 16, 0, p, q, p, r, None) == _lib.FFT3D_E_INVALID_ARG
    assert f(16, 16, 16, 1, p + 8, q, p, r, None) == _lib.FFT3D_E_ALIGNMENT
    assert f(16, 16, 16, 1, p, q, p, r + 4, None) == _lib.FFT3D_E_ALIGNMENT
    assert f(16, 14, 16, 1, p, q, p, r, None) == _lib.FFT3D_E_UNSUPPORTED_SIZE
    assert f(256, 256, 16, 1, p, q, p, r, None) == _lib.FFT3D_E_UNSUPPORTED_SIZE
    assert f(16, 8, 16, 1, p, q, p, r, None) == _lib.FFT3D_E_UNSUPPORTED
    # partial sums beyond the fixed array: 511 grids of 128 x 128 rows
    assert f(128, 128, 1, 511, p, q, p, r, None) == _lib.FFT3D_E_SCRATCH
    torch.cuda.synchronize()
