"""Batched/mixed form: heterogeneous grids in one persistent launch."""
import json
import os

import numpy as np
import pytest

import oracle
import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 5e-6
SCHEDULES = [(t, c) for t in (1024, 512) for c in (1, 2, 4, 8)]


def rel(a, b):
    a = np.asarray(a, np.complex128).ravel()
    b = np.asarray(b, np.complex128).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(scope="module")
def F(tmp_path_factory):
    import paper_2006_08435_amd as m
    # keep tuning-cache lookups away from the user's home cache
    os.environ["FFT3D_TUNE_CACHE"] = str(tmp_path_factory.mktemp("tc") / "tune.json")
    return m


def inputs(groups, seed0):
    out = []
    for g, (n, b) in enumerate(groups):
        out.append(np.stack([workloads.sphere_grid(n, seed0 + 97 * g + j) for j in range(b)]))
    return out


def run(plan, xs):
    ins = [torch.from_numpy(x).cuda() for x in xs]
    outs = plan.exec(ins)
    torch.cuda.synchronize()
    return [o.cpu().numpy() for o in outs]


@pytest.mark.parametrize("direction", [-1, 1])
def test_mixed_small_groups_match_oracle(F, direction):
    groups = [(64, 5), (48, 2), (32, 3), (100, 1), (24, 4)]
    xs = inputs(groups, 11)
    plan = F.PlanMany(groups, direction)
    got = run(plan, xs)
    for (n, b), x, y in zip(groups, xs, got):
        for j in range(b):
            ref = oracle.fft3d(x[j].astype(np.complex128), direction)
            assert rel(y[j], ref) <= TOL, (n, j)
    from paper_2006_08435_amd import _lib
    assert _lib.lib().fft3d_plan_check(plan.handle) == 0


def test_every_schedule_gives_identical_results(F):
    groups = [(64, 3), (72, 1), (48, 2), (128, 1)]
    xs = inputs(groups, 5)
    plan = F.PlanMany(groups, -1)
    ref = None
    for t, c in SCHEDULES:
        plan.set_schedule(t, c)
        got = run(plan, xs)
        if ref is None:
            ref = got
            for (n, b), x, y in zip(groups, xs, got):
                assert rel(y[0], oracle.fft3d(x[0].astype(np.complex128), -1)) <= TOL
        else:
            for a, b in zip(ref, got):
                assert np.array_equal(a, b), (t, c)
    from paper_2006_08435_amd import _lib
    assert _lib.lib().fft3d_plan_check(plan.handle) == 0


def test_grouped_mode(F):
    """threads = 0: each group's plane and z passes as plain launches; same
    transform as the persistent kernel (to rounding: other kernels)."""
    groups = [(64, 3), (72, 1), (48, 2), (128, 1)]
    xs = inputs(groups, 7)
    plan = F.PlanMany(groups, -1)
    plan.set_schedule(1024, 2)
    pers = run(plan, xs)
    plan.set_schedule(0, 1)
    assert "mode=grouped" in plan.describe()
    got = run(plan, xs)
    for (n, b), x, y, z in zip(groups, xs, got, pers):
        for j in range(b):
            assert rel(y[j], oracle.fft3d(x[j].astype(np.complex128), -1)) <= TOL
        assert rel(y, z) <= 1e-6


def test_hybrid_mode(F):
    """threads < 0: a group with enough planes to fill the device runs its
    plain passes (bit-identical to grouped mode), the others share one
    persistent launch (bit-identical to the persistent mode's results for
    those grids)."""
    groups = [(64, 64), (72, 1), (48, 2), (100, 1)]
    xs = inputs(groups, 9)
    plan = F.PlanMany(groups, 1)
    plan.set_schedule(0, 1)
    grouped = run(plan, xs)
    plan.set_schedule(1024, 2)
    pers = run(plan, xs)
    plan.set_schedule(-1024, 2)
    d = plan.describe()
    assert "mode=hybrid grouped=64^3x64 " in d and "threads=1024 chunk=2" in d, d
    got = run(plan, xs)
    assert np.array_equal(got[0], grouped[0])
    for a, b in zip(got[1:], pers[1:]):
        assert np.array_equal(a, b)
    for (n, b), x, y in zip(groups, xs, got):
        for j in (0, b - 1):
            assert rel(y[j], oracle.fft3d(x[j].astype(np.complex128), 1)) <= TOL, (n, j)
    from paper_2006_08435_amd import _lib
    assert _lib.lib().fft3d_plan_check(plan.handle) == 0


@pytest.mark.parametrize("groups,mode", [([(48, 2), (36, 3)], "grouped=none"), ([(64, 64)], "items=0")])
def test_hybrid_degenerate_splits(F, groups, mode):
    """All groups small: the persistent launch alone; all big: plain passes
    alone (no persistent launch)."""
    xs = inputs(groups, 19)
    plan = F.PlanMany(groups, -1)
    plan.set_schedule(-512, 4)
    assert mode in plan.describe(), plan.describe()
    got = run(plan, xs)
    plan.set_schedule(0 if mode == "items=0" else 512, 4)
    want = run(plan, xs)
    for a, b in zip(got, want):
        assert np.array_equal(a, b)


def test_matches_plain_per_grid_execs(F):
    groups = [(96, 2), (60, 3)]
    xs = inputs(groups, 21)
    plan = F.PlanMany(groups, 1)
    got = run(plan, xs)
    for (n, b), x, y in zip(groups, xs, got):
        for j in range(b):
            plain = F.ifftn(torch.from_numpy(x[j]).cuda()).cpu().numpy()
            assert rel(y[j], plain) <= 1e-6


def test_inplace_and_repeat(F):
    groups = [(64, 6), (48, 3)]
    xs = inputs(groups, 31)
    plan = F.PlanMany(groups, -1)
    first = run(plan, xs)
    ins = [torch.from_numpy(x).cuda() for x in xs]
    for _ in range(10):
        bufs = [t.clone() for t in ins]
        plan.exec(bufs, bufs)
    torch.cuda.synchronize()
    for a, b in zip(first, bufs):
        assert np.array_equal(a, b.cpu().numpy())


@pytest.mark.parametrize("threads,chunk,groups", [(1024, 2, [(64, 4), (80, 1), (36, 2)]),
                                                  (0, 1, [(64, 4), (80, 1), (36, 2)]),
                                                  (-1024, 2, [(64, 48), (80, 1), (36, 2)])])
def test_graph_capture_replays_match_eager(F, threads, chunk, groups):
    xs = inputs(groups, 41)
    plan = F.PlanMany(groups, -1)
    plan.set_schedule(threads, chunk)
    ins = [torch.from_numpy(x).cuda() for x in xs]
    eager = [o.clone() for o in plan.exec(ins)]
    outs = [torch.empty_like(t) for t in ins]
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            plan.exec(ins, outs, stream=s)
    torch.cuda.current_stream().wait_stream(s)
    for r in range(5):
        for o in outs:
            o.zero_()
        g.replay()
        torch.cuda.synchronize()
        for a, b in zip(eager, outs):
            assert torch.equal(a, b), r
        plan.exec(ins)              # eager work between replays
        torch.cuda.synchronize()


@pytest.mark.parametrize("direction", [-1, 1])
def test_group_schedule_variants_match_oracle(F, direction):
    """Every radix order and z-tile width of the plain passes (the tuner's
    candidates) against the oracle, on sizes whose alternative order swaps
    two radices (48, 120) or splits the length another way (36 = 9x4,
    64 = 16x4, 100 = 4x5x5: three stages)."""
    groups = [(48, 2), (120, 1), (36, 2), (64, 2), (100, 1)]
    xs = inputs(groups, 77)
    refs = [[oracle.fft3d(x[j].astype(np.complex128), direction) for j in range(b)]
            for (n, b), x in zip(groups, xs)]
    plan = F.PlanMany(groups, direction)
    plan.set_schedule(0, 1)   # grouped mode: every group runs its plain passes
    radices = {0: "16x3,8x15,6x6,8x8,10x10", 1: "3x16,15x8,9x4,16x4,4x5x5"}
    for order, lines in [(1, 64), (0, 32), (1, 32), (0, 64)]:
        for g in range(len(groups)):
            plan.set_group_schedule(g, order, lines)
        d = plan.describe()
        assert "radix=" + radices[order] in d and "zlines=" + ",".join([str(lines)] * len(groups)) in d, d
        got = run(plan, xs)
        for (n, b), y, r in zip(groups, got, refs):
            for j in range(b):
                assert rel(y[j], r[j]) <= TOL, (n, order, lines, j, rel(y[j], r[j]))
    from paper_2006_08435_amd import _lib
    L = _lib.lib()
    assert L.fft3d_plan_set_group_schedule(plan.handle, 5, 0, 64) == _lib.FFT3D_E_INVALID_ARG
    assert L.fft3d_plan_set_group_schedule(plan.handle, 0, 2, 64) == _lib.FFT3D_E_INVALID_ARG
    assert L.fft3d_plan_set_group_schedule(plan.handle, 0, 0, 16) == _lib.FFT3D_E_INVALID_ARG


def test_tuner_and_cache(F, tmp_path, monkeypatch):
    cache = tmp_path / "tune.json"
    monkeypatch.setenv("FFT3D_TUNE_CACHE", str(cache))
    monkeypatch.setenv("FFT3D_TUNE", "1")
    groups = [(64, 4), (48, 1)]
    p1 = F.PlanMany(groups, -1)
    assert "tuned" in p1.describe()
    d = json.loads(cache.read_text())
    (key, val), = d.items()
    assert val["threads"] in (0, 512, 1024, -512, -1024) and 1 <= val["chunk"] <= 8 and val["ms"] > 0
    # per group: the radix order and z-tile width the tuner chose
    kinds = [int(v) for v in val["radix"].split(",")]
    zl = [int(v) for v in val["zlines"].split(",")]
    assert len(kinds) == len(groups) and set(kinds) <= {0, 2} and len(zl) == len(groups) and set(zl) <= {32, 64}
    monkeypatch.delenv("FFT3D_TUNE")
    p2 = F.PlanMany(groups, -1)            # read back from the cache
    assert "tuned" in p2.describe()
    if val["threads"] == 0:
        assert "mode=grouped" in p2.describe()
    else:
        assert "threads=%d chunk=%d" % (abs(val["threads"]), val["chunk"]) in p2.describe()
        assert ("mode=hybrid" in p2.describe()) == (val["threads"] < 0)
    cache.write_text("{ this is not json")  # a corrupt cache falls back to the default
    p3 = F.PlanMany(groups, -1)
    assert "default" in p3.describe()
    xs = inputs(groups, 51)
    for a, b in zip(run(p1, xs), run(p3, xs)):
        if val["threads"] <= 0:             # other kernels (for some groups): equal to rounding
            assert rel(a, b) <= 1e-6
        else:
            assert np.array_equal(a, b)


def test_mixed_grid_workload(F):
    """256 grids of 64^3 plus one each of 48^3, 72^3, 96^3, 100^3, 120^3."""
    groups = [(64, 256)] + [(n, 1) for n in workloads.MIXED_SIZES]
    xs = [np.stack([workloads.sphere_grid(64, workloads.SEED_BATCH64 + j) for j in range(256)])]
    xs += [workloads.sphere_grid(n, workloads.SEED_MIXED + n)[None] for n in workloads.MIXED_SIZES]
    plan = F.PlanMany(groups, 1)
    got = run(plan, xs)
    worst = 0.0
    for (n, b), x, y in zip(groups, xs, got):
        for j in ([0, 77, 255] if b > 1 else [0]):
            r = rel(y[j], oracle.fft3d(x[j].astype(np.complex128), 1))
            worst = max(worst, r)
    assert worst <= TOL, worst
    # every 64^3 grid: Parseval against its input
    e_in = np.sum(np.abs(xs[0].astype(np.complex128)) ** 2, axis=(1, 2, 3))
    e_out = np.sum(np.abs(got[0].astype(np.complex128)) ** 2, axis=(1, 2, 3))
    assert np.all(np.abs(e_out - 64 ** 3 * e_in) <= 1e-5 * 64 ** 3 * e_in)
