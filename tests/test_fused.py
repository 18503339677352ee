"""The persistent fused kernel (plane items + z-slab items with per-grid
dependency counters): parity, repeatability, health check, graph replay.

The fused scheme is selected with FFT3D_FUSED=1 at plan time (the default for
cubic grids is the two-pass plane + z schedule); this module sets it for its
own plans and restores the environment afterwards."""
import os
import subprocess
import sys

import numpy as np
import pytest

import oracle
import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 5e-6


def rel(a, b):
    a = np.asarray(a, np.complex128).ravel()
    b = np.asarray(b, np.complex128).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(scope="module")
def fft3d():
    import paper_2006_08435_amd as m
    old = os.environ.get("FFT3D_FUSED")
    os.environ["FFT3D_FUSED"] = "1"
    yield m
    if old is None:
        del os.environ["FFT3D_FUSED"]
    else:
        os.environ["FFT3D_FUSED"] = old


@pytest.mark.parametrize("n,batch", [(128, 5), (64, 9), (96, 3), (48, 17), (120, 2), (100, 1), (18, 40), (125, 1)])
def test_fused_batches_match_oracle(fft3d, n, batch):
    x = workloads.uniform_grid(n, 31 * n + batch, batch=batch)
    plan = fft3d.Plan(n, n, n, batch, "fp32", -1)
    assert plan.describe().startswith("fused"), plan.describe()
    xt = torch.from_numpy(x).cuda()
    y = plan.exec(xt)
    torch.cuda.synchronize()
    got = y.cpu().numpy()
    for j in sorted({0, batch // 2, batch - 1}):
        ref = oracle.fft3d(x[j].astype(np.complex128), -1)
        assert rel(got[j], ref) <= TOL, (n, batch, j)
    from paper_2006_08435_amd import _lib
    assert _lib.lib().fft3d_plan_check(plan.handle) == 0


def test_repeated_execs_are_identical(fft3d):
    """Counters self-reset: many back-to-back execs give bitwise-equal output."""
    n, batch = 64, 12
    x = torch.from_numpy(workloads.uniform_grid(n, 3, batch=batch)).cuda()
    plan = fft3d.Plan(n, n, n, batch, "fp32", 1)
    first = plan.exec(x).clone()
    out = torch.empty_like(x)
    for _ in range(20):
        plan.exec(x, out)
    torch.cuda.synchronize()
    assert torch.equal(first, out)
    from paper_2006_08435_amd import _lib
    assert _lib.lib().fft3d_plan_check(plan.handle) == 0


def test_fused_inplace(fft3d):
    n, batch = 128, 3
    x = workloads.uniform_grid(n, 8, batch=batch)
    plan = fft3d.Plan(n, n, n, batch, "fp32", -1)
    a = plan.exec(torch.from_numpy(x).cuda())
    b = torch.from_numpy(x).cuda()
    plan.exec(b, b)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_fused_matches_two_kernel_path(fft3d):
    """Without FFT3D_FUSED the planner picks the separate plane and z kernels
    (run in a child process so the variable is read at plan time)."""
    n, batch = 96, 4
    x = workloads.uniform_grid(n, 4, batch=batch)
    plan = fft3d.Plan(n, n, n, batch, "fp32", -1)
    y = plan.exec(torch.from_numpy(x).cuda()).cpu().numpy()
    code = ("import sys, numpy as np, torch; sys.path.insert(0, %r);"
            "import workloads, paper_2006_08435_amd as f;"
            "x = workloads.uniform_grid(%d, 4, batch=%d);"
            "p = f.Plan(%d, %d, %d, %d, 'fp32', -1); assert p.describe().startswith('plane'), p.describe();"
            "np.save(sys.argv[1], p.exec(torch.from_numpy(x).cuda()).cpu().numpy())"
            % (os.path.dirname(os.path.dirname(os.path.abspath(__file__))), n, batch, n, n, n, batch))
    out = os.path.join("/tmp", "fused_ref_%d.npy" % os.getpid())
    env = dict(os.environ)
    env.pop("FFT3D_FUSED", None)
    subprocess.run([sys.executable, "-c", code, out], check=True, env=env, timeout=300)
    z = np.load(out)
    os.remove(out)
    assert rel(y, z) <= 1e-6


@pytest.mark.parametrize("fused", [True, False])
def test_graph_capture_replays_match_eager(fft3d, fused, monkeypatch):
    if not fused:
        monkeypatch.delenv("FFT3D_FUSED")
    n, batch = 64, 8
    x = torch.from_numpy(workloads.uniform_grid(n, 6, batch=batch)).cuda()
    fwd = fft3d.Plan(n, n, n, batch, "fp32", -1)
    inv = fft3d.Plan(n, n, n, batch, "fp32", 1)
    mid = torch.empty_like(x)
    out = torch.empty_like(x)
    eager_mid = fwd.exec(x).clone()
    eager_out = inv.exec(eager_mid).clone()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            fwd.exec(x, mid, stream=s)
            inv.exec(mid, out, stream=s)
    torch.cuda.current_stream().wait_stream(s)
    for r in range(5):
        mid.zero_()
        out.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(mid, eager_mid), r
        assert torch.equal(out, eager_out), r
        # eager work between replays
        fwd.exec(x, mid)
        torch.cuda.synchronize()
        assert torch.equal(mid, eager_mid), r
    from paper_2006_08435_amd import _lib
    assert _lib.lib().fft3d_plan_check(fwd.handle) == 0
    assert _lib.lib().fft3d_plan_check(inv.handle) == 0


@pytest.mark.parametrize("n,batch", [(128, 16), (64, 16), (96, 8), (48, 24), (128, 10), (32, 3)])
def test_xcd_local_variant(fft3d, n, batch, monkeypatch):
    """FFT3D_FUSED=2: every XCD owns whole grids (its own queue); checked
    against the oracle, for repeats, and by the drained-queue health check."""
    monkeypatch.setenv("FFT3D_FUSED", "2")
    x = workloads.uniform_grid(n, 7 * n + batch, batch=batch)
    plan = fft3d.Plan(n, n, n, batch, "fp32", 1)
    assert "xcd_queues=" in plan.describe() and "xcd_queues=0" not in plan.describe(), plan.describe()
    xt = torch.from_numpy(x).cuda()
    first = plan.exec(xt).clone()
    out = torch.empty_like(xt)
    for _ in range(5):
        plan.exec(xt, out)
    torch.cuda.synchronize()
    assert torch.equal(first, out)
    got = first.cpu().numpy()
    for j in sorted({0, batch // 2, batch - 1}):
        assert rel(got[j], oracle.fft3d(x[j].astype(np.complex128), 1)) <= TOL, (n, batch, j)
    from paper_2006_08435_amd import _lib
    assert _lib.lib().fft3d_plan_check(plan.handle) == 0
