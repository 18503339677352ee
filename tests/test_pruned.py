"""Pruned transforms for a sphere cutoff (fft3d_plan_set_cutoff), on the GPU.

The input of a plane-wave inverse transform vanishes outside a sphere
|G|^2 < r2 in frequency space, and only the sphere is kept of a forward
transform (Section I's operator evaluation, with the cutoff restriction of
Section III).  The pruned inverse skips the planes and rows that hold only
zeros; the pruned forward skips the stores, and the z-lines, that do not
reach the sphere.  What they compute is still the DFT of Eq. (1).  Bars:

* agreement with the dense plan on the same input (the inverse: everywhere;
  the forward: inside the sphere): both schedules apply the same butterflies
  in the same order to the same values, the pruned one only substitutes
  literal zeros for loads of zeros and drops stores.  The compiler may
  contract a few multiply-adds of the pruned kernels into FMAs differently,
  so the bar is FP32 rounding: every element within 16 ulp of the largest
  magnitude.  The inverse kernels are in fact bit-identical as compiled and
  the tests say so (==);
* the FP32 tolerance (relative L2 <= 5e-6) against the FP64 oracle.
"""

import numpy as np
import pytest

import oracle
import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 5e-6
INVERSE, FORWARD = 1, -1


@pytest.fixture(scope="module")
def fft3d():
    import paper_2006_08435_amd as m
    assert torch.cuda.is_available()
    return m


def sphere_mask(nx, nz, r2):
    gz = workloads.signed_freq(nz)[:, None, None]
    gy = workloads.signed_freq(nx)[None, :, None]
    gx = workloads.signed_freq(nx)[None, None, :]
    return (gx * gx + gy * gy + gz * gz) < r2


def dense_input(nx, nz, batch, seed):
    if nx == nz:
        return workloads.uniform_grid(nx, seed, batch=batch)
    rng = np.random.default_rng(seed)
    x = rng.uniform(-1, 1, (batch, nz, nx, nx)) + 1j * rng.uniform(-1, 1, (batch, nz, nx, nx))
    return x.astype(np.complex64)


def sphere_input(nx, nz, batch, r2, seed):
    """Uniform complex values inside Gx^2+Gy^2+Gz^2 < r2, exact zeros outside."""
    x = dense_input(nx, nz, batch, seed)
    return np.where(sphere_mask(nx, nz, r2)[None], x, np.complex64(0)).astype(np.complex64)


def assert_rounding_close(ref, got):
    """Every element within 16 FP32 ulp of the largest magnitude."""
    scale = float(ref.abs().max())
    err = float((ref - got).abs().max())
    assert err <= 16 * 2.0 ** -23 * scale, (err, scale)


def dense_and_pruned(fft3d, x, r2, inplace=False, direction=INVERSE):
    b, nz, ny, nx = x.shape
    dense = fft3d.Plan(nx, ny, nz, b, "fp32", direction)
    pruned = fft3d.Plan(nx, ny, nz, b, "fp32", direction)
    pruned.set_cutoff(r2)
    xt = torch.from_numpy(np.ascontiguousarray(x)).cuda()
    ref = dense.exec(xt)
    if inplace:
        got = xt.clone()
        pruned.exec(got, got)
    else:
        got = pruned.exec(xt)
    torch.cuda.synchronize()
    return ref, got, pruned


CASES = [
    # (nx, nz, batch, r2)
    (24, 24, 3, (24 / 4.0) ** 2),
    (32, 32, 2, (32 / 4.0) ** 2),
    (32, 32, 2, 0.5),            # only G = 0
    (32, 32, 1, 3 * 32 ** 2),    # every point inside: the dense schedule's work
    (45, 45, 2, (45 / 4.0) ** 2),
    (64, 64, 2, (64 / 4.0) ** 2),
    (64, 64, 1, (64 / 2.0) ** 2),
    (75, 75, 1, 200.0),
    (96, 96, 1, (96 / 4.0) ** 2),
    (125, 125, 1, (125 / 4.0) ** 2),
    (128, 128, 2, (128 / 4.0) ** 2),
    (48, 30, 2, 100.0),          # nz != nx
    (16, 16, 4, 16.0),           # sizes that use the whole-cube kernel densely
    (12, 5, 2, 9.0),
]


@pytest.mark.parametrize("nx,nz,batch,r2", CASES)
def test_equals_dense_inverse(fft3d, nx, nz, batch, r2):
    x = sphere_input(nx, nz, batch, r2, 7000 + nx + nz)
    ref, got, plan = dense_and_pruned(fft3d, x, r2)
    assert "k_plane_pruned" in plan.describe()
    assert torch.equal(ref, got), float((ref - got).abs().max())


@pytest.mark.parametrize("nx,nz,batch,r2", CASES)
def test_forward_equals_dense_inside_sphere(fft3d, nx, nz, batch, r2):
    x = dense_input(nx, nz, batch, 7500 + nx + nz)
    ref, got, plan = dense_and_pruned(fft3d, x, r2, direction=FORWARD)
    assert "k_plane_pruned" in plan.describe()
    m = torch.from_numpy(np.broadcast_to(sphere_mask(nx, nz, r2)[None], x.shape).copy()).cuda()
    assert_rounding_close(ref[m], got[m])


@pytest.mark.parametrize("nx,nz,batch,r2", [(32, 32, 2, 64.0), (128, 128, 1, 1024.0), (48, 30, 2, 100.0)])
def test_in_place(fft3d, nx, nz, batch, r2):
    x = sphere_input(nx, nz, batch, r2, 7100 + nx)
    ref, got, _ = dense_and_pruned(fft3d, x, r2, inplace=True)
    assert torch.equal(ref, got)
    x = dense_input(nx, nz, batch, 7150 + nx)
    ref, got, _ = dense_and_pruned(fft3d, x, r2, inplace=True, direction=FORWARD)
    m = torch.from_numpy(np.broadcast_to(sphere_mask(nx, nz, r2)[None], x.shape).copy()).cuda()
    assert_rounding_close(ref[m], got[m])


@pytest.mark.parametrize("nx,r2", [(32, 64.0), (60, 225.0), (64, 256.0)])
def test_against_oracle(fft3d, nx, r2):
    x = sphere_input(nx, nx, 2, r2, 7200 + nx)
    _, got, _ = dense_and_pruned(fft3d, x, r2)
    want = oracle.fft3d(x.astype(np.complex128), sign=+1)
    g = got.cpu().numpy().astype(np.complex128)
    for j in range(x.shape[0]):
        err = np.linalg.norm(g[j] - want[j]) / np.linalg.norm(want[j])
        assert err <= TOL, (j, err)


@pytest.mark.parametrize("nx,r2", [(32, 64.0), (60, 225.0), (64, 256.0)])
def test_forward_against_oracle(fft3d, nx, r2):
    x = dense_input(nx, nx, 2, 7250 + nx)
    _, got, _ = dense_and_pruned(fft3d, x, r2, direction=FORWARD)
    want = oracle.fft3d(x.astype(np.complex128), sign=-1)
    m = sphere_mask(nx, nx, r2)
    g = got.cpu().numpy().astype(np.complex128)
    for j in range(x.shape[0]):
        err = np.linalg.norm(g[j][m] - want[j][m]) / np.linalg.norm(want[j][m])
        assert err <= TOL, (j, err)


def test_round_trip_on_sphere(fft3d):
    """Pruned inverse then pruned forward returns N^3 times the sphere."""
    n, r2 = 48, 144.0
    c = sphere_input(n, n, 2, r2, 7600)
    inv = fft3d.Plan(n, n, n, 2, "fp32", INVERSE)
    fwd = fft3d.Plan(n, n, n, 2, "fp32", FORWARD)
    inv.set_cutoff(r2)
    fwd.set_cutoff(r2)
    ct = torch.from_numpy(c).cuda()
    back = fwd.exec(inv.exec(ct))
    torch.cuda.synchronize()
    m = sphere_mask(n, n, r2)
    got = back.cpu().numpy()[:, m] / n ** 3
    want = c[:, m]
    assert np.linalg.norm(got - want) / np.linalg.norm(want) <= TOL


def test_sphere_workload_config_cutoff(fft3d):
    """The plane-wave workload's own recipe (radius N/4) at 32 x 128^3."""
    n, b = 128, 32
    x = workloads.sphere_batch(n, [workloads.SEED_BATCH128 + j for j in range(b)])
    ref, got, plan = dense_and_pruned(fft3d, x, (n / 4.0) ** 2)
    assert "zplanes=63" in plan.describe()
    assert torch.equal(ref, got)


@pytest.mark.parametrize("direction", [INVERSE, FORWARD])
def test_passes_compose_to_exec(fft3d, direction):
    n, r2 = 64, 256.0
    x = sphere_input(n, n, 2, r2, 7300)
    plan = fft3d.Plan(n, n, n, 2, "fp32", direction)
    plan.set_cutoff(r2)
    lib = fft3d._lib.lib()
    assert lib.fft3d_plan_passes(plan.handle) == 2
    xt = torch.from_numpy(x).cuda()
    a = plan.exec(xt)
    b = torch.empty_like(xt)
    s = torch.cuda.current_stream().cuda_stream
    assert lib.fft3d_exec_pass(plan.handle, 0, xt.data_ptr(), b.data_ptr(), s) == 0
    assert lib.fft3d_exec_pass(plan.handle, 1, b.data_ptr(), b.data_ptr(), s) == 0
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_clear_restores_dense(fft3d):
    n = 64
    plan = fft3d.Plan(n, n, n, 1, "fp32", INVERSE)
    dense_desc = plan.describe()
    plan.set_cutoff(100.0)
    assert "cutoff_r2=100" in plan.describe()
    plan.set_cutoff(0.0)
    assert plan.describe() == dense_desc
    x = workloads.uniform_grid(n, 7400, batch=1)   # dense input: no zeros
    xt = torch.from_numpy(x).cuda()
    ref = fft3d.Plan(n, n, n, 1, "fp32", INVERSE).exec(xt)
    got = plan.exec(xt)
    torch.cuda.synchronize()
    assert torch.equal(ref, got)


def test_rejections(fft3d):
    lib = fft3d._lib.lib()
    axes = fft3d.Plan(32, 24, 32, 1, "fp32", INVERSE)
    assert lib.fft3d_plan_set_cutoff(axes.handle, 10.0) == -7
    q = fft3d.Plan(64, 64, 64, 1, "fp16", INVERSE)
    assert lib.fft3d_plan_set_cutoff(q.handle, 10.0) == -7
    inv = fft3d.Plan(32, 32, 32, 1, "fp32", INVERSE)
    assert lib.fft3d_plan_set_cutoff(inv.handle, float("nan")) == -1
    many = fft3d.PlanMany([(32, 2)], direction=INVERSE)
    assert lib.fft3d_plan_set_cutoff(many.handle, 10.0) == -7
