"""Sanitizer tier (CPU only): the oracle and the library's host code built
with AddressSanitizer and UndefinedBehaviorSanitizer, and the CPU tests that
exercise them run against those builds in a child process (the sanitizer
runtime has to be preloaded into the interpreter, which is not
instrumented).  Device code is not instrumented.  Skips when a sanitizer
runtime or compiler is absent."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE_SRC = os.path.join(ROOT, "oracle", "oracle.c")
GCC_SAN = ["-O1", "-g", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-fno-fast-math", "-ffp-contract=off",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]


def _runtime(cmd):
    try:
        p = subprocess.run(cmd, capture_output=True, text=True, timeout=60).stdout.strip()
    except (OSError, subprocess.SubprocessError):
        return None
    return p if os.path.isabs(p) and os.path.exists(p) else None


def gcc_asan():
    return _runtime(["gcc", "-print-file-name=libasan.so"]) if shutil.which("gcc") else None


def clang_asan():
    clang = "/opt/rocm/llvm/bin/clang"
    return _runtime([clang, "-print-file-name=libclang_rt.asan-x86_64.so"]) if os.path.exists(clang) else None


def run_child(args, env_extra, preload):
    env = dict(os.environ)
    env.update(env_extra)
    env["LD_PRELOAD"] = preload
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0:exitcode=86"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1:exitcode=87"
    env["CUDA_VISIBLE_DEVICES"] = ""
    env["HIP_VISIBLE_DEVICES"] = ""
    return subprocess.run([sys.executable] + args, cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)


def build_oracle(src_text, out):
    src = out + ".c"
    with open(src, "w") as f:
        f.write(src_text)
    subprocess.run(["gcc"] + GCC_SAN + [src, "-o", out, "-lm"], check=True)
    return out


def test_oracle_pins_under_asan_ubsan(tmp_path):
    """Every oracle pin passes with the oracle instrumented."""
    rt = gcc_asan()
    if rt is None:
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    lib = build_oracle(open(ORACLE_SRC).read(), str(tmp_path / "liboracle_san.so"))
    r = run_child(["-m", "pytest", "-q", "-p", "no:cacheprovider", "tests/test_oracle.py"],
                  {"FFT3D_ORACLE_LIB": lib}, rt)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert "passed" in r.stdout


def test_sanitized_oracle_catches_a_planted_overflow(tmp_path):
    """Positive control: the energy buffer made too small by one factor 2
    (a planted mistake in a copy of the oracle) is reported."""
    rt = gcc_asan()
    if rt is None:
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    text = open(ORACLE_SRC).read()
    start = text.index("int oracle_energy(")
    body = text[start:]
    alloc = "malloc(sizeof(double) * 2 * vol * batch)"
    assert alloc in body
    planted = text[:start] + body.replace(alloc, "malloc(sizeof(double) * vol * batch)", 1)
    lib = build_oracle(planted, str(tmp_path / "liboracle_planted.so"))
    code = ("import numpy as np, oracle\n"
            "c = np.ones((1, 4, 4, 4), np.complex128)\n"
            "V = np.ones((4, 4, 4))\n"
            "oracle.energy(c, V, want_grad=False)\n")
    r = run_child(["-c", code], {"FFT3D_ORACLE_LIB": lib}, rt)
    assert r.returncode != 0 and "AddressSanitizer" in r.stderr, r.stderr[-2000:]


def test_library_host_code_under_asan_ubsan(tmp_path):
    """The C-ABI argument checks, planning errors and symbol table of
    libfft3d.so with its host logic (fft3d_api.cpp, fft3d_many.cpp,
    fft3d_noalloc.hip) instrumented."""
    rt = clang_asan()
    if rt is None:
        pytest.skip("clang's AddressSanitizer runtime is not installed")
    from paper_2006_08435_amd import build
    try:
        lib = build.build_host_sanitized(str(tmp_path / "hostsan"))
    except (OSError, RuntimeError) as e:
        pytest.skip("sanitized host build unavailable: %s" % str(e)[:200])
    r = run_child(["-m", "pytest", "-q", "-p", "no:cacheprovider", "-m", "not gpu", "tests/test_abi.py"],
                  {"FFT3D_LIB_PATH": lib}, rt)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert "passed" in r.stdout
