"""Pins that tie the FP64 oracle to facts fixed by the paper and by mathematics.

Each ``pin_*`` function raises AssertionError when the oracle disagrees.  They
are run directly by ``test_oracle.py`` and again, against builds of the oracle
with planted mistakes, by ``test_oracle_mutants.py`` (every planted mistake
must trip at least one pin).

Sources of truth (none of them is the oracle itself):
* hand-derived worked examples of Eq. (1) (``tests/golden``);
* closed forms: impulse -> constant, constant -> DC spike, shifted impulse ->
  phase ramp, plane wave -> spike;
* invariants: forward(inverse) = N^3 I, Parseval, linearity, shift theorem,
  Hermitian symmetry of the transform of real data, separability (any axis
  order gives the same result);
* independent library routines as witnesses: numpy.fft (pocketfft, also its
  real transforms rfftn / irfftn), numpy's float16 conversion, torch's
  bfloat16 conversion, torch autograd.
"""
from __future__ import annotations

import json
import os

import numpy as np

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
SMALL_SIZES = [1, 2, 3, 4, 5, 6, 8, 9, 10, 12, 15, 16]
NONCUBIC = [(2, 3, 5), (4, 6, 5), (8, 3, 10), (5, 1, 3)]   # (nx, ny, nz)


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
    a = np.asarray(a, dtype=np.complex128).ravel()
    b = np.asarray(b, dtype=np.complex128).ravel()
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def rand_grid(shape, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def numpy_ref(a, sign):
    """numpy.fft witness for Eq. (1) (sign -1) and its unnormalised inverse."""
    axes = (-3, -2, -1)
    if sign == -1:
        return np.fft.fftn(a, axes=axes)
    n = a.shape[-1] * a.shape[-2] * a.shape[-3]
    return np.fft.ifftn(a, axes=axes) * n


def _grid_coords(nz, ny, nx):
    z = np.arange(nz)[:, None, None]
    y = np.arange(ny)[None, :, None]
    x = np.arange(nx)[None, None, :]
    return z, y, x


# ---------------------------------------------------------------- Eq. (1) ----

def pin_golden(fn=None):
    """Hand-derived worked examples of Eq. (1)."""
    fn = fn or oracle.dft3d_naive
    with open(os.path.join(HERE, "golden", "eq1_worked_examples.json")) as f:
        spec = json.load(f)
    env = {"sqrt": np.sqrt, "cos": np.cos, "sin": np.sin, "pi": np.pi}
    for case in spec["cases"]:
        nz, ny, nx = case["shape"]
        z, y, x = _grid_coords(nz, ny, nx)
        loc = dict(env, x=x, y=y, z=z)
        re = np.broadcast_to(eval(case["input_re"], {}, loc), (nz, ny, nx))
        im = np.broadcast_to(eval(case["input_im"], {}, loc), (nz, ny, nx))
        f = (re + 1j * im).astype(np.complex128)
        expect = np.zeros((nz, ny, nx), dtype=np.complex128)
        for idx, er, ei in case["expected_nonzero"]:
            expect[tuple(idx)] = eval(er, {}, env) + 1j * eval(ei, {}, env)
        got = fn(f, case.get("sign", -1))
        assert np.max(np.abs(got - expect)) < 1e-12, (case["name"], got, expect)


def pin_closed_forms(fn=None, shapes=((4, 4, 4), (3, 5, 2), (6, 2, 5))):
    """Impulse, constant, shifted impulse, plane wave -- both signs."""
    fn = fn or oracle.dft3d_naive
    for (nx, ny, nz) in shapes:
        vol = nx * ny * nz
        z, y, x = _grid_coords(nz, ny, nx)
        kz, ky, kx = _grid_coords(nz, ny, nx)
        for sign in (-1, 1):
            d = np.zeros((nz, ny, nx), complex)
            d[0, 0, 0] = 1.0
            assert np.max(np.abs(fn(d, sign) - 1.0)) < 1e-13, "impulse"
            c = np.full((nz, ny, nx), 0.75 - 0.5j)
            F = fn(c, sign)
            e = np.zeros_like(F)
            e[0, 0, 0] = (0.75 - 0.5j) * vol
            assert np.max(np.abs(F - e)) < 1e-12 * vol, "constant"
            x0, y0, z0 = nx - 1, ny // 2, min(1, nz - 1)
            s = np.zeros((nz, ny, nx), complex)
            s[z0, y0, x0] = 1.0
            ramp = np.exp(sign * 2j * np.pi * (kx * x0 / nx + ky * y0 / ny + kz * z0 / nz))
            assert np.max(np.abs(fn(s, sign) - ramp)) < 1e-12, "shifted impulse"
            k0 = (nx // 2, max(ny - 1, 0), nz // 3)
            wave = np.exp(-sign * 2j * np.pi * (x * k0[0] / nx + y * k0[1] / ny + z * k0[2] / nz))
            spike = np.zeros((nz, ny, nx), complex)
            spike[k0[2], k0[1], k0[0]] = vol
            assert np.max(np.abs(fn(wave, sign) - spike)) < 1e-11 * vol, "plane wave"


def pin_naive_vs_numpy():
    for shape in [(n, n, n) for n in (1, 2, 3, 4, 5, 6, 8)] + NONCUBIC:
        nx, ny, nz = shape
        a = rand_grid((2, nz, ny, nx), 11 + nx + 7 * ny + 31 * nz)
        for sign in (-1, 1):
            assert rel(oracle.dft3d_naive(a, sign), numpy_ref(a, sign)) < 1e-13, (shape, sign)


# ------------------------------------------------------------ the FFT (O2) ----

def pin_fft_vs_naive():
    shapes = [(n, n, n) for n in SMALL_SIZES] + NONCUBIC
    for (nx, ny, nz) in shapes:
        a = rand_grid((nz, ny, nx), 100 + nx * 13 + ny * 7 + nz)
        for sign in (-1, 1):
            r = rel(oracle.fft3d(a, sign), oracle.dft3d_naive(a, sign))
            assert r < 1e-13, ((nx, ny, nz), sign, r)


def pin_fft_vs_numpy():
    for n in smooth_sizes(128) + [7, 11, 13, 49, 77]:
        v = rand_grid((n,), 500 + n)
        assert rel(oracle.fft1d(v, -1), np.fft.fft(v)) < 1e-13, n
        assert rel(oracle.fft1d(v, 1), np.fft.ifft(v) * n) < 1e-13, n
    for shape in [(48, 48, 48), (64, 64, 64), (100, 100, 100), (30, 20, 12), (128, 16, 8)]:
        nx, ny, nz = shape
        a = rand_grid((nz, ny, nx), sum(shape))
        for sign in (-1, 1):
            assert rel(oracle.fft3d(a, sign), numpy_ref(a, sign)) < 1e-13, (shape, sign)


def pin_invariants():
    for (nx, ny, nz) in [(8, 8, 8), (12, 10, 9), (16, 5, 6), (4, 6, 5)]:
        vol = nx * ny * nz
        f = rand_grid((2, nz, ny, nx), vol)
        g = rand_grid((2, nz, ny, nx), vol + 1)
        F = oracle.fft3d(f, -1)
        # forward then inverse = vol * identity (both orders)
        assert rel(oracle.fft3d(F, 1), vol * f) < 1e-14
        assert rel(oracle.fft3d(oracle.fft3d(f, 1), -1), vol * f) < 1e-14
        # Parseval
        assert abs(np.vdot(F, F).real - vol * np.vdot(f, f).real) < 1e-12 * vol * np.vdot(f, f).real
        # linearity
        al, be = 0.3 - 1.2j, -2.0 + 0.5j
        assert rel(oracle.fft3d(al * f + be * g, -1), al * F + be * oracle.fft3d(g, -1)) < 1e-14
        # shift theorem with a cyclic shift by (ax, ay, az)
        ax, ay, az = 1, ny - 1, 2 % nz
        fs = np.roll(f, shift=(az, ay, ax), axis=(1, 2, 3))
        kz, ky, kx = _grid_coords(nz, ny, nx)
        ph = np.exp(-2j * np.pi * (kx * ax / nx + ky * ay / ny + kz * az / nz))
        assert rel(oracle.fft3d(fs, -1), ph[None] * F) < 1e-13
        # Hermitian symmetry for real input: F[-k] = conj F[k]
        r = oracle.fft3d(f.real.astype(complex), -1)
        neg = np.roll(np.flip(r, axis=(1, 2, 3)), shift=(1, 1, 1), axis=(1, 2, 3))
        assert rel(neg, np.conj(r)) < 1e-14
        # separability: every axis order gives the same 3D transform
        for order in [(2, 1, 0), (1, 2, 0), (0, 2, 1)]:
            assert rel(oracle.fft3d(f, -1, order=order), F) < 1e-14, order


# ------------------------------------------------------- scaled 16-bit data ----

def pin_fp16_rounding():
    """Round-to-nearest-even into binary16 matches numpy's float16 cast."""
    rng = np.random.default_rng(7)
    vals = np.concatenate([
        rng.standard_normal(3000) * 2.0 ** rng.integers(-26, 17, 3000),
        np.array([0.0, -0.0, 1.0, 65504.0, 65519.0, 65520.0, 2.0 ** -24, 2.0 ** -25,
                  3 * 2.0 ** -25, 2.0 ** -14, 1 + 2.0 ** -11, 1 + 3 * 2.0 ** -11,
                  -(1 + 2.0 ** -11), 2048 + 1, 2048 + 3, 1e6]),
    ]).astype(np.float32)
    want = vals.astype(np.float16).view(np.uint16)
    got = np.array([oracle.round_fp16(float(v)) for v in vals], dtype=np.uint16)
    assert np.array_equal(got, want), np.nonzero(got != want)
    back = np.array([oracle.fp16_value(int(h)) for h in want])
    assert np.array_equal(back, want.view(np.float16).astype(np.float64))


def pin_bf16_rounding():
    """Round-to-nearest-even into bfloat16 matches torch's bfloat16 cast."""
    import torch
    rng = np.random.default_rng(8)
    vals = np.concatenate([
        rng.standard_normal(3000) * 2.0 ** rng.integers(-130, 120, 3000),
        np.array([0.0, 1.0, 1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8, -(1 + 2.0 ** -8),
                  2.0 ** -133, 3.0e38, 1e-40]),
    ]).astype(np.float32)
    t = torch.from_numpy(vals).to(torch.bfloat16)
    want = t.view(torch.int16).numpy().view(np.uint16)
    got = np.array([oracle.round_bf16(float(v)) for v in vals], dtype=np.uint16)
    assert np.array_equal(got, want), np.nonzero(got != want)
    back = np.array([oracle.bf16_value(int(h)) for h in want])
    assert np.array_equal(back, t.to(torch.float64).numpy())


def pin_q16_rule():
    """Exponent rule and error bound of the scaled 16-bit encoding."""
    rng = np.random.default_rng(9)
    rows = (rng.standard_normal((64, 40)) + 1j * rng.standard_normal((64, 40)))
    rows *= 2.0 ** rng.integers(-60, 60, (64, 1))
    rows[3] = 0.0                        # all-zero row: exponent 0
    rows[5] = 0.0
    rows[5, 7] = 2.0 ** 14               # row maximum exactly 2^14: exponent 0
    rows[6] = 0.0
    rows[6, 1] = -1j * 2.0 ** 15         # maximum on the imaginary part: exponent 1
    a = rows.astype(np.complex64)
    for fmt, frac in ((oracle.FMT_FP16, 10), (oracle.FMT_BF16, 7)):
        payload, e = oracle.q16_encode(a, fmt)
        assert e[3] == 0 and e[5] == 0 and e[6] == 1
        m = np.maximum(np.abs(a.real), np.abs(a.imag)).max(axis=1).astype(np.float64)
        nz = m > 0
        scaled = m[nz] * 2.0 ** (-e[nz].astype(np.float64))
        assert np.all(scaled >= 2.0 ** 14) and np.all(scaled < 2.0 ** 15)
        dec = oracle.q16_decode(payload, e, fmt)
        err = np.abs(dec - a.astype(np.complex128)).max(axis=1)
        # RNE: each component off by at most half a quantum of the row's scale
        bound = 2.0 ** (e.astype(np.float64) + 14 - frac - 1)
        assert np.all(err <= bound * np.sqrt(2))
        if fmt == oracle.FMT_FP16:
            # binary16 payload equals numpy's float16 cast of the scaled value
            sc = (a.view(np.float32).reshape(64, 80).astype(np.float64)
                  * 2.0 ** (-e[:, None].astype(np.float64))).astype(np.float32)
            assert np.array_equal(payload.reshape(64, 80), sc.astype(np.float16).view(np.uint16))


# -------------------------------------------------------------- the energy ----

def pin_energy():
    """E and its gradient: numpy witness, exact central differences, autograd."""
    import torch
    nx, ny, nz, b = 6, 5, 4, 3
    c = rand_grid((b, nz, ny, nx), 77)
    V = np.random.default_rng(78).uniform(-1, 2, (nz, ny, nx))
    E, psi, grad = oracle.energy(c, V, want_psi=True, want_grad=True)
    vol = nx * ny * nz
    psi_np = np.fft.ifftn(c, axes=(-3, -2, -1)) * vol
    assert rel(psi, psi_np) < 1e-13
    assert abs(E - float(np.sum(V * np.abs(psi_np) ** 2))) < 1e-12 * abs(E)
    # E is quadratic in c, so the central difference is exact for any step
    rng = np.random.default_rng(79)
    for eps in (1e-3, 0.7):
        d = rng.standard_normal(c.shape) + 1j * rng.standard_normal(c.shape)
        Ep, _, _ = oracle.energy(c + eps * d, V, want_grad=False)
        Em, _, _ = oracle.energy(c - eps * d, V, want_grad=False)
        fd = (Ep - Em) / (2 * eps)
        lin = float(np.real(np.vdot(grad, d)))
        assert abs(fd - lin) < 1e-9 * (abs(lin) + abs(E) * 1e-3), (eps, fd, lin)
    # torch autograd (float64, CPU) as an independent witness of the convention
    ct = torch.from_numpy(c.copy()).requires_grad_(True)
    pt = torch.fft.ifftn(ct, dim=(-3, -2, -1), norm="forward")
    Et = (torch.from_numpy(V) * (pt.real ** 2 + pt.imag ** 2)).sum()
    Et.backward()
    assert rel(grad, ct.grad.numpy()) < 1e-12


# ------------------------------------------------------------ real grids ----

REAL_SHAPES = [(8, 6, 5), (2, 3, 4), (12, 12, 5), (10, 1, 3), (6, 4, 1)]   # (nx, ny, nz)


def pin_real():
    """r2c / c2r: numpy's rfftn / irfftn as witnesses, a plane-wave closed
    form, and the round trip c2r(r2c(f)) = NxNyNz f."""
    for i, (nx, ny, nz) in enumerate(REAL_SHAPES):
        vol = nx * ny * nz
        f = np.random.default_rng(300 + i).standard_normal((2, nz, ny, nx))
        H = oracle.r2c3d(f)
        assert H.shape == (2, nz, ny, nx // 2 + 1)
        assert rel(H, np.fft.rfftn(f, axes=(-3, -2, -1))) < 1e-13, (nx, ny, nz)
        back = oracle.c2r3d(H, nx)
        assert np.max(np.abs(back - vol * f)) < 1e-12 * vol * np.max(np.abs(f)), (nx, ny, nz)
        # an arbitrary (not Hermitian) half spectrum: the imaginary parts of
        # the kx = 0 and kx = nx/2 entries must not contribute
        h = rand_grid((2, nz, ny, nx // 2 + 1), 400 + i)
        want = np.fft.irfftn(h, s=(nz, ny, nx), axes=(-3, -2, -1)) * vol
        got = oracle.c2r3d(h, nx)
        assert np.max(np.abs(got - want)) < 1e-12 * np.max(np.abs(want)), (nx, ny, nz)
    # plane wave cos(2 pi (a x/nx + b y/ny + c z/nz)): half spectrum vol/2 at (c, b, a)
    nx, ny, nz, a, b, c = 12, 10, 6, 5, 3, 4
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    f = np.cos(2 * np.pi * (a * x / nx + b * y / ny + c * z / nz))
    H = oracle.r2c3d(f)
    want = np.zeros((nz, ny, nx // 2 + 1), np.complex128)
    want[c, b, a] = nx * ny * nz / 2
    assert np.max(np.abs(H - want)) < 1e-10


def pin_apply_potential():
    """forward(V inverse(c)): numpy witness, constant potential, self-adjointness
    (<a, H b> = <H a, b> for real V), and half the energy gradient."""
    nx, ny, nz, b = 6, 4, 5, 2
    c = rand_grid((b, nz, ny, nx), 500)
    V = np.random.default_rng(501).uniform(-1, 2, (nz, ny, nx))
    vol = nx * ny * nz
    H = oracle.apply_potential(c, V)
    want = np.fft.fftn(V * np.fft.ifftn(c, axes=(-3, -2, -1)) * vol, axes=(-3, -2, -1))
    assert rel(H, want) < 1e-13
    const = oracle.apply_potential(c, np.full((nz, ny, nx), 0.75))
    assert rel(const, 0.75 * vol * c) < 1e-13
    a = rand_grid((nz, ny, nx), 502)
    d = rand_grid((nz, ny, nx), 503)
    lhs = np.vdot(a, oracle.apply_potential(d, V))
    rhs = np.vdot(oracle.apply_potential(a, V), d)
    assert abs(lhs - rhs) < 1e-10 * abs(lhs)
    _, _, grad = oracle.energy(c, V, want_grad=True)
    assert rel(H, grad / 2) < 1e-13


def pin_density():
    """rho = sum f_n |psi_n|^2: numpy witness, the integral sum_r rho =
    N^3 sum_n f_n sum_G |c_n|^2 (unnormalised inverse), one plane wave."""
    nx, ny, nz, b = 6, 5, 4, 3
    c = rand_grid((b, nz, ny, nx), 600)
    f = np.array([2.0, 1.5, 0.25])
    vol = nx * ny * nz
    rho = oracle.density(c, f)
    psi = np.fft.ifftn(c, axes=(-3, -2, -1)) * vol
    assert np.max(np.abs(rho - np.einsum("b,bzyx->zyx", f, np.abs(psi) ** 2))) < 1e-10 * np.max(rho)
    total = vol * float(np.sum(f[:, None, None, None] * np.abs(c) ** 2))
    assert abs(rho.sum() - total) < 1e-10 * total
    one = np.zeros((1, nz, ny, nx), np.complex128)
    one[0, 1, 2, 3] = 2.0 - 1.0j                 # |psi| = |c| everywhere
    assert np.allclose(oracle.density(one, [0.5]), 0.5 * 5.0, rtol=1e-14, atol=0)


ALL_PINS = [pin_golden, pin_closed_forms, pin_naive_vs_numpy, pin_fft_vs_naive,
            pin_fft_vs_numpy, pin_invariants, pin_fp16_rounding, pin_bf16_rounding,
            pin_q16_rule, pin_energy, pin_real, pin_apply_potential, pin_density]
