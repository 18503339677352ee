"""Plant plausible mistakes in the oracle (on the CPU) and check a pin trips.

Each mutant is a one-line textual change to oracle/oracle.c, compiled into a
temporary library; the pins of ``oracle_pins`` run against it and at least one
must fail.  This shows the pins constrain every part of the oracle: twiddle
signs and indices, strides of the axis passes, the brute-force sum, the
16-bit rounding and exponent rule, and the energy gradient.
"""
import pytest

import oracle
import oracle_pins as P

MUTANTS = {
    "complex product sign": ("im += t[2 * q] * c[1] + t[2 * q + 1] * c[0];",
                             "im += t[2 * q] * c[1] - t[2 * q + 1] * c[0];"),
    "combine drops s*m": ("long e = ((long)q * kk) % n;", "long e = ((long)q * k) % n;"),
    "y stride uses ny": ("(axis == 1 ? (long)nx : (long)nx * ny)",
                         "(axis == 1 ? (long)ny : (long)nx * ny)"),
    "y pencil base uses nz": ("base = z * (long)nx * ny + x;", "base = z * (long)nx * nz + x;"),
    "naive drops a term": ("re += fr * tr - fi * ti;", "re += fr * tr;"),
    "naive wrong index": ("wy + 2 * (((long)y * ky) % ny)", "wy + 2 * (((long)y * kx) % ny)"),
    "root table ignores sign": ("w[2 * e + 1] = (double)sign * sin(a);",
                                "w[2 * e + 1] = sin(a);"),
    "gradient drops factor 2": ("p[2 * (b * vol + i)] *= 2.0 * V[i];",
                                "p[2 * (b * vol + i)] *= V[i];"),
    "gradient uses inverse": ("err = oracle_fft3d(nx, ny, nz, batch, -1, p, grad);",
                              "err = oracle_fft3d(nx, ny, nz, batch, +1, p, grad);"),
    "psi uses forward": ("int err = oracle_fft3d(nx, ny, nz, batch, +1, c, p);",
                         "int err = oracle_fft3d(nx, ny, nz, batch, -1, c, p);"),
    "exponent off by one": ("e = ilogb(m) - 14;", "e = ilogb(m) - 15;"),
    "ties round up": ("return fmod(f, 2.0) == 0.0 ? f : f + 1.0;", "return f + 1.0;"),
    "no subnormal quantum": ("if (e < emin) e = emin;", "(void)emin;"),
    "c2r drops factor 2": ("v += 2.0 * (H[2 * k]", "v += (H[2 * k]"),
    "c2r Nyquist sign": ("((x & 1) ? -H[2 * (nx / 2)] : H[2 * (nx / 2)])", "H[2 * (nx / 2)]"),
    "c2r sin sign": ("- H[2 * k + 1] * w[2 * e + 1]", "+ H[2 * k + 1] * w[2 * e + 1]"),
    "c2r skips z": ("if (!err) err = axis_pass(h, ny, nz, batch, +1, 2, t);", "(void)0;"),
    "apply uses forward first": ("oracle_fft3d(nx, ny, nz, batch, inverse, c, p);",
                                 "oracle_fft3d(nx, ny, nz, batch, forward, c, p);"),
    "apply skips V imag": ("                p[2 * (b * vol + i) + 1] *= V[i];\n            }\n        err = oracle_fft3d(nx, ny, nz, batch, forward, p, out);",
                           "            }\n        err = oracle_fft3d(nx, ny, nz, batch, forward, p, out);"),
    "density uses forward": ("oracle_fft3d(nx, ny, nz, batch, inverse_sign, c, p);",
                             "oracle_fft3d(nx, ny, nz, batch, -inverse_sign, c, p);"),
    "density drops occupation": ("rho[i] += occ[b] * (re * re + im * im);", "rho[i] += (re * re + im * im);"),
    "density keeps last orbital": ("rho[i] += occ[b] * (re * re + im * im);", "rho[i] = occ[b] * (re * re + im * im);"),
    "r2c wrong half": ("out[2 * (r * h + k)] = full[2 * (r * nx + k)];",
                       "out[2 * (r * h + k)] = full[2 * (r * nx + (nx - k) % nx)];"),
}


# Each mutant runs in a child process: a planted indexing mistake (a wrong
# stride, say) can write outside the oracle's buffers, and that must not
# corrupt the test runner's own heap.  The child loads the mutant, runs the
# pins until one fails, prints its name and leaves without running any
# destructor.
_CHILD = r"""
import os, sys
sys.path.insert(0, {tests!r})
sys.path.insert(0, {root!r})
import oracle
import oracle_pins as P
with oracle.variant({lib!r}):
    for pin in P.ALL_PINS:
        try:
            pin()
        except Exception as e:
            print("CAUGHT", pin.__name__, type(e).__name__, flush=True)
            os._exit(0)
print("MISSED", flush=True)
os._exit(0)
"""


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(name, tmp_path):
    import os
    import subprocess
    import sys
    old, new = MUTANTS[name]
    src = oracle.source_text()
    assert src.count(old) == 1, "mutation site not found: %s" % name
    lib = oracle.build_variant(src.replace(old, new), str(tmp_path / "libmutant.so"))
    here = os.path.dirname(os.path.abspath(__file__))
    code = _CHILD.format(tests=here, root=os.path.dirname(here), lib=lib)
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert "CAUGHT" in r.stdout, "no pin caught mutant %r (exit %d): %s %s" % (name, r.returncode, r.stdout,
                                                                            r.stderr[-500:])
