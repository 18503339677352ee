"""Seeded randomized properties of the FP32 transform on the GPU: random
2*3*5-smooth shapes up to 128 per side (square planes and general shapes,
so the plane + z and the three-axis schedules both run), random batches of
1 to 7, both signs.  Every case against the FP64 oracle, in place equal to
out of place bit for bit, the same exec on a second stream equal bit for
bit, and a graph replay equal to the eager result bit for bit."""
import numpy as np
import pytest

import oracle
import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 5e-6


def smooth(n):
    for p in (2, 3, 5):
        while n % p == 0:
            n //= p
    return n == 1


SIZES = [n for n in range(1, 129) if smooth(n)]


def cases(count=24, seed=20261):
    rng = np.random.default_rng(seed)
    out = []
    for k in range(count):
        nx = int(rng.choice(SIZES))
        ny = nx if k % 2 == 0 else int(rng.choice(SIZES))
        nz = int(rng.choice(SIZES))
        # keep each case to at most 2^20 points per grid so the oracle stays fast
        while nx * ny * nz > (1 << 20):
            nz = int(rng.choice([s for s in SIZES if s <= nz // 2] or [1]))
        out.append((nx, ny, nz, int(rng.integers(1, 8)), int(rng.choice([-1, 1]))))
    return out


def rel(a, b):
    a = np.asarray(a, np.complex128).ravel()
    b = np.asarray(b, np.complex128).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(scope="module")
def F():
    import paper_2006_08435_amd as m
    return m


@pytest.mark.parametrize("nx,ny,nz,batch,direction", cases())
def test_random_shape_properties(F, nx, ny, nz, batch, direction):
    x = workloads.uniform_grid((nx, ny, nz), 31 * nx + 7 * ny + nz + batch, batch=batch)
    plan = F.Plan(nx, ny, nz, batch, "fp32", direction)
    xt = torch.from_numpy(x).cuda()
    out = plan.exec(xt)
    torch.cuda.synchronize()
    ref = oracle.fft3d(x.astype(np.complex128), direction)
    got = out.cpu().numpy()
    for j in range(batch):
        assert rel(got[j], ref[j]) <= TOL, (nx, ny, nz, batch, direction, j, rel(got[j], ref[j]))
    # in place
    ip = xt.clone()
    plan.exec(ip, ip)
    # another stream
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    o2 = torch.empty_like(xt)
    with torch.cuda.stream(s):
        plan.exec(xt, o2, stream=s)
    torch.cuda.current_stream().wait_stream(s)
    # graph replay
    o3 = torch.zeros_like(xt)
    g = torch.cuda.CUDAGraph()
    s2 = torch.cuda.Stream()
    s2.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s2):
        with torch.cuda.graph(g, stream=s2):
            plan.exec(xt, o3, stream=s2)
    torch.cuda.current_stream().wait_stream(s2)
    g.replay()
    torch.cuda.synchronize()
    assert torch.equal(ip, out) and torch.equal(o2, out) and torch.equal(o3, out)
