"""Reduced-precision form: scaled 16-bit storage (binary16 / bfloat16 payload,
per-row power-of-two exponent), FP32 arithmetic, radix-16 on the matrix
cores.  Bars: conversions bit-exact against the oracle's encoder; transforms
within relative L2 2e-3 of the FP64 oracle applied to the dequantized input."""
import os

import numpy as np
import pytest

import oracle
import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL16 = 2e-3
FMT = {"fp16": oracle.FMT_FP16, "bf16": oracle.FMT_BF16}


def rel(a, b):
    a = np.asarray(a, np.complex128).ravel()
    b = np.asarray(b, np.complex128).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(scope="module")
def F():
    import paper_2006_08435_amd as m
    return m


def split(buf, shape):
    """scaled16 byte buffer -> (uint16 payload [..., 2], int8 exps) numpy views."""
    n = int(np.prod(shape))
    b = buf.cpu().numpy()
    pay = b[:4 * n].view(np.uint16).reshape(tuple(shape) + (2,))
    ex = b[4 * n:].view(np.int8).reshape(tuple(shape[:-1]))
    return pay, ex


def join(pay, ex):
    return torch.from_numpy(np.concatenate([pay.reshape(-1).view(np.uint8), ex.reshape(-1).view(np.uint8)])).cuda()


def rows_fixture():
    rng = np.random.default_rng(17)
    a = (rng.standard_normal((96, 40)) + 1j * rng.standard_normal((96, 40)))
    a *= 2.0 ** rng.integers(-40, 40, (96, 1))
    a[2] = 0
    a[3] = 0
    a[3, 5] = 2.0 ** 14
    a[4] = 0
    a[4, 0] = -1j * 2.0 ** 15
    a[5] *= 1e-30
    a[6, ::2] *= 1e-6       # wide dynamic range inside one row
    return a.astype(np.complex64)


@pytest.mark.parametrize("prec", ["fp16", "bf16"])
def test_quantize_bit_exact(F, prec):
    a = rows_fixture()
    buf = F.quantize(torch.from_numpy(a).cuda(), prec)
    torch.cuda.synchronize()
    pay, ex = split(buf, a.shape)
    rp, re_ = oracle.q16_encode(a, FMT[prec])
    assert np.array_equal(ex, re_)
    assert np.array_equal(pay, rp)


@pytest.mark.parametrize("prec", ["fp16", "bf16"])
def test_dequantize_bit_exact(F, prec):
    a = rows_fixture()
    rp, re_ = oracle.q16_encode(a, FMT[prec])
    got = F.dequantize(join(rp, re_), a.shape, prec).cpu().numpy()
    want = oracle.q16_decode(rp, re_, FMT[prec])
    assert np.array_equal(got.astype(np.complex128), want)


def check_storage_rule(pay, ex, prec):
    """Every row of a scaled16 array obeys the storage rule: with m the
    largest |re| or |im| of the row's payload (the 16-bit values, exponent
    not applied), m == 0 has exponent 0; otherwise 2^14 <= m <= 2^15 (2^15
    when the row maximum rounded up to it), unless the exponent is clamped
    at -128.  A row maximum taken over the wrong lanes or rows breaks it."""
    v = oracle.q16_decode(pay, np.zeros_like(ex), FMT[prec])
    m = np.maximum(np.abs(v.real), np.abs(v.imag)).max(axis=-1)
    e = ex.astype(np.int64)
    zero = m == 0
    assert np.all(e[zero] == 0)
    assert np.all(m[~zero] <= 2.0 ** 15)
    assert np.all((m >= 2.0 ** 14) | (e == -128) | zero)


def run_q16(F, x, prec, direction, inplace=False):
    b, n = x.shape[0], x.shape[-1]
    xt = torch.from_numpy(x).cuda()
    qin = F.quantize(xt, prec)
    plan = F.Plan(n, n, n, b, prec, direction)
    if inplace:
        plan.exec(qin, qin)
        out = qin
    else:
        out = plan.exec(qin)
    torch.cuda.synchronize()
    pin, ein = split(qin if not inplace else F.quantize(xt, prec), x.shape)
    pout, eout = split(out, x.shape)
    return plan, pin, ein, pout, eout


@pytest.mark.parametrize("n", [16, 32, 48, 64, 80, 96, 128])
@pytest.mark.parametrize("prec", ["fp16", "bf16"])
@pytest.mark.parametrize("direction", [1, -1])
def test_transform_within_bound(F, n, prec, direction):
    b = 2 if n <= 64 else 1
    x = np.stack([workloads.sphere_grid(n, 900 + n + j) for j in range(b)])
    plan, pin, ein, pout, eout = run_q16(F, x, prec, direction)
    engine = "MFMA" if os.environ.get("FFT3D_Q16_MFMA") == "1" else "VALU"   # radix-16 engine chosen at plan time
    assert "scaled16" in plan.describe() and "radix-16 on " + engine in plan.describe()
    xin = oracle.q16_decode(pin, ein, FMT[prec])        # the input IS the 16-bit data
    got = oracle.q16_decode(pout, eout, FMT[prec])
    ref = oracle.fft3d(xin, direction)
    for j in range(b):
        r = rel(got[j], ref[j])
        assert r <= TOL16, (n, prec, direction, j, r)
    check_storage_rule(pout, eout, prec)


@pytest.mark.parametrize("n", [32, 64, 96, 128])
@pytest.mark.parametrize("prec", ["fp16", "bf16"])
@pytest.mark.parametrize("direction", [1, -1])
def test_plane_pass_intermediate(F, n, prec, direction):
    """The plane pass alone (fft3d_exec_pass 0): its intermediate, always
    scaled FP16, is the 2D DFT over (y, x) of every z-plane of the
    dequantized input, and obeys the storage rule row by row."""
    from paper_2006_08435_amd import _lib
    b = 2 if n <= 64 else 1
    x = np.stack([workloads.sphere_grid(n, 700 + n + j) for j in range(b)])
    xt = torch.from_numpy(x).cuda()
    qin = F.quantize(xt, prec)
    plan = F.Plan(n, n, n, b, prec, direction)
    mid = torch.empty_like(qin)
    s = torch.cuda.current_stream().cuda_stream
    assert _lib.lib().fft3d_exec_pass(plan.handle, 0, qin.data_ptr(), mid.data_ptr(), s) == 0
    torch.cuda.synchronize()
    pin, ein = split(qin, x.shape)
    pm, em = split(mid, x.shape)
    check_storage_rule(pm, em, "fp16")
    xin = oracle.q16_decode(pin, ein, FMT[prec]).reshape(b * n, 1, n, n)
    ref = oracle.fft3d(xin, direction).reshape(x.shape)
    got = oracle.q16_decode(pm, em, oracle.FMT_FP16)
    for j in range(b):
        r = rel(got[j], ref[j])
        assert r <= TOL16, (n, prec, direction, j, r)


@pytest.mark.parametrize("engine", ["0", "1"])
@pytest.mark.parametrize("prec", ["fp16", "bf16"])
@pytest.mark.parametrize("n", [64, 128])
def test_power_of_two_scale_equivariance(F, engine, prec, n, monkeypatch):
    """Scaling the input by 2^k (exponents only) scales every stage exactly:
    the output payload is the same bit for bit and every nonzero row's
    exponent moves by k, with either radix-16 engine (the matrix-core one
    folds row exponents into its DFT matrix, relative to the largest
    exponent of the rows that are not all zero)."""
    monkeypatch.setenv("FFT3D_Q16_MFMA", engine)
    x = workloads.sphere_grid(n, 4242 + n)[None]
    p0, e0, outs = None, None, {}
    rp, re_ = oracle.q16_encode(x, FMT[prec])
    for k in (0, 40, -40):
        plan = F.Plan(n, n, n, 1, prec, 1)
        ek = np.where(np.any(rp & 0x7FFF, axis=(-2, -1)), re_.astype(np.int64) + k, 0).astype(np.int8)
        out = plan.exec(join(rp, ek))
        torch.cuda.synchronize()
        outs[k] = split(out, x.shape)
    pay0, ex0 = outs[0]
    nzrow = np.any(pay0 & 0x7FFF, axis=(-2, -1))
    for k in (40, -40):
        pay, ex = outs[k]
        assert np.array_equal(pay, pay0), (engine, prec, n, k)
        assert np.array_equal(ex[nzrow].astype(np.int64), ex0[nzrow].astype(np.int64) + k), (engine, prec, n, k)
        assert np.all(ex[~nzrow] == 0)


def test_inplace_matches_out_of_place(F):
    x = np.stack([workloads.sphere_grid(64, 5 + j) for j in range(3)])
    _, _, _, p1, e1 = run_q16(F, x, "fp16", 1)
    _, _, _, p2, e2 = run_q16(F, x, "fp16", 1, inplace=True)
    assert np.array_equal(p1, p2) and np.array_equal(e1, e2)


def test_matches_fp32_path(F):
    """The 16-bit transform equals the FP32 transform of the same (dequantized)
    input to the same bound."""
    n = 96
    x = workloads.sphere_grid(n, 77)[None]
    _, pin, ein, pout, eout = run_q16(F, x, "fp16", -1)
    xin = oracle.q16_decode(pin, ein, oracle.FMT_FP16).astype(np.complex64)
    y32 = F.fftn(torch.from_numpy(xin).cuda()).cpu().numpy()
    assert rel(oracle.q16_decode(pout, eout, oracle.FMT_FP16), y32) <= TOL16


def batch_128(B=32, n=128):
    x = np.empty((B, n, n, n), np.complex64)
    for j in range(B):
        x[j] = workloads.sphere_grid(n, workloads.SEED_BATCH128 + j)
    return x


def check_every_grid(pin, ein, pout, eout, prec, direction):
    """Every grid of the batch against the FP64 oracle on its dequantized
    input, element by element (relative L2 per grid)."""
    worst = 0.0
    for j in range(pin.shape[0]):
        xin = oracle.q16_decode(pin[j:j + 1], ein[j:j + 1], FMT[prec])
        got = oracle.q16_decode(pout[j:j + 1], eout[j:j + 1], FMT[prec])
        r = rel(got, oracle.fft3d(xin, direction))
        assert r <= TOL16, (prec, direction, j, r)
        worst = max(worst, r)
    check_storage_rule(pout, eout, prec)
    return worst


@pytest.mark.parametrize("prec", ["fp16", "bf16"])
def test_batch_32x128(F, prec, monkeypatch):
    """32 grids of 128^3 (the large precision-form workload) with the default
    vector-ALU radix-16 engine, every grid, both directions."""
    monkeypatch.delenv("FFT3D_Q16_MFMA", raising=False)
    x = batch_128()
    for direction in (1, -1):
        plan, pin, ein, pout, eout = run_q16(F, x, prec, direction)
        assert "radix-16 on VALU" in plan.describe()
        check_every_grid(pin, ein, pout, eout, prec, direction)


@pytest.mark.parametrize("n", [16, 64, 128])
@pytest.mark.parametrize("prec", ["fp16", "bf16"])
@pytest.mark.parametrize("direction", [1, -1])
def test_mfma_engine_within_bound(F, n, prec, direction, monkeypatch):
    """The same transform with the radix-16 stage as a DFT-matrix product on
    the matrix cores (FFT3D_Q16_MFMA=1), both signs of the DFT matrix."""
    monkeypatch.setenv("FFT3D_Q16_MFMA", "1")
    x = np.stack([workloads.sphere_grid(n, 300 + n + j) for j in range(2)])
    plan, pin, ein, pout, eout = run_q16(F, x, prec, direction)
    assert "radix-16 on MFMA" in plan.describe()
    xin = oracle.q16_decode(pin, ein, FMT[prec])
    got = oracle.q16_decode(pout, eout, FMT[prec])
    assert rel(got, oracle.fft3d(xin, direction)) <= TOL16
    check_storage_rule(pout, eout, prec)


@pytest.mark.parametrize("prec", ["fp16", "bf16"])
def test_mfma_batch_32x128(F, prec, monkeypatch):
    """The matrix-core engine on the full 32 x 128^3 batch: these are the
    launches with streaming loads that only a batch of 32 MB or more takes;
    every grid, both directions."""
    monkeypatch.setenv("FFT3D_Q16_MFMA", "1")
    x = batch_128()
    for direction in (1, -1):
        plan, pin, ein, pout, eout = run_q16(F, x, prec, direction)
        assert "radix-16 on MFMA" in plan.describe()
        check_every_grid(pin, ein, pout, eout, prec, direction)


def bf16_bits(a):
    """bfloat16 bit patterns of float32 values, rounded to nearest even
    (finite values)."""
    u = np.ascontiguousarray(a, np.float32).view(np.uint32).astype(np.uint64)
    return ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16)


@pytest.mark.parametrize("engine", ["0", "1"])
@pytest.mark.parametrize("n", [64, 128])
def test_bf16_payloads_any_range(F, engine, n, monkeypatch):
    """bfloat16 input as a caller may hand it over, not in the storage rule's
    normal form: zero exponents with rows 2^-60 ... 2^60 in size, and plain
    payloads whose row exponents lie up to 130 apart (rows more than 100 below
    the largest, which the matrix-core engine drops, weigh less than FP32
    rounding).  Both radix-16 engines against the oracle on the same input."""
    monkeypatch.setenv("FFT3D_Q16_MFMA", engine)
    rng = np.random.default_rng(4400 + n)
    x = workloads.sphere_grid(n, 4400 + n)[None]
    xs = (x * (2.0 ** rng.integers(-60, 61, size=x.shape[:-1]))[..., None]).astype(np.complex64)
    variants = [
        (np.stack([bf16_bits(xs.real), bf16_bits(xs.imag)], axis=-1), np.zeros(x.shape[:-1], np.int8)),
        (np.stack([bf16_bits(x.real), bf16_bits(x.imag)], axis=-1),
         rng.integers(-110, 21, size=x.shape[:-1]).astype(np.int8)),
    ]
    for direction in (1, -1):
        for pay, ex in variants:
            plan = F.Plan(n, n, n, 1, "bf16", direction)
            out = plan.exec(join(pay, ex))
            torch.cuda.synchronize()
            pout, eout = split(out, x.shape)
            xin = oracle.q16_decode(pay, ex, oracle.FMT_BF16)
            got = oracle.q16_decode(pout, eout, oracle.FMT_BF16)
            assert rel(got, oracle.fft3d(xin, direction)) <= TOL16, (engine, n, direction)
            check_storage_rule(pout, eout, "bf16")
