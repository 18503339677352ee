"""HIP-graph capture of the pruned, real-grid and local-potential entry points.

Each form is captured once into a graph and replayed several times, with
the program's own eager work between replays; every replay must equal the
eager result element for element (no form records memset nodes or
allocates during execution).
"""
import numpy as np
import pytest

import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    import paper_2006_08435_amd as m
    assert torch.cuda.is_available()
    return m


def capture_and_check(fn, outs, eager_between):
    """fn(stream) enqueues the work writing `outs`; compare replays to eager."""
    cur = torch.cuda.current_stream()
    fn(cur)
    torch.cuda.synchronize()
    ref = [o.clone() for o in outs]
    s = torch.cuda.Stream()
    s.wait_stream(cur)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            fn(s)
    cur.wait_stream(s)
    for r in range(4):
        for o in outs:
            o.zero_()
        g.replay()
        torch.cuda.synchronize()
        for a, b in zip(ref, outs):
            assert torch.equal(a, b), r
        eager_between()
        torch.cuda.synchronize()


def test_pruned_inverse_forward_graph(F):
    n, b, r2 = 64, 2, 256.0
    c = np.stack([workloads.sphere_grid(n, 12000 + j) for j in range(b)])
    inv = F.Plan(n, n, n, b, "fp32", 1)
    fwd = F.Plan(n, n, n, b, "fp32", -1)
    inv.set_cutoff(r2)
    fwd.set_cutoff(r2)
    ct = torch.from_numpy(c).cuda()
    psi = torch.empty_like(ct)
    back = torch.zeros_like(ct)   # points outside the sphere are never written: start (and replay) from zeros
    packed = torch.empty((b, inv.sphere_points), dtype=torch.complex64, device="cuda")
    work = torch.empty_like(ct)

    def fn(s):
        inv.exec(ct, psi, stream=s)
        fwd.exec(psi, back, stream=s)
        work.copy_(psi)
        fwd.exec_packed(work, packed, stream=s)

    capture_and_check(fn, [psi, back, packed], lambda: inv.exec(ct))


def test_real_graph(F):
    n, b = 48, 3
    f = np.random.default_rng(12100).uniform(-1, 1, (b, n, n, n)).astype(np.float32)
    r2c = F.RealPlan(n, n, n, b, -1)
    c2r = F.RealPlan(n, n, n, b, 1)
    ft = torch.from_numpy(f).cuda()
    half = torch.empty(r2c.half_shape, dtype=torch.complex64, device="cuda")
    scratch = torch.empty_like(half)
    back = torch.empty_like(ft)

    def fn(s):
        r2c.exec(ft, half, stream=s)
        scratch.copy_(half)
        c2r.exec(scratch, back, stream=s)

    capture_and_check(fn, [half, back], lambda: r2c.exec(ft))


@pytest.mark.parametrize("cutoff", [None, 576.0])
def test_apply_potential_graph(F, cutoff):
    n, b = 96, 2
    c = np.stack([workloads.sphere_grid(n, 12200 + j) for j in range(b)])
    V = workloads.smooth_potential(n, 12299)
    plan = F.Plan(n, n, n, b, "fp32", 1)
    if cutoff:
        plan.set_cutoff(cutoff)
    ct = torch.from_numpy(c).cuda()
    Vt = torch.from_numpy(V).cuda()
    out = torch.zeros_like(ct)   # with a cutoff, points outside the sphere are never written
    E = torch.zeros((), dtype=torch.float64, device="cuda")

    def fn(s):
        plan.apply_potential(ct, Vt, out=out, E=E, stream=s)

    capture_and_check(fn, [out, E], lambda: plan.apply_potential(ct, Vt))
