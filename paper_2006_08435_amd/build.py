"""Build libfft3d.so (HIP, gfx950) in-tree.

Every HIP/C++ source under csrc/ is compiled by hipcc for gfx950 into
_build/, in parallel, and linked into paper_2006_08435_amd/libfft3d.so.
Packed-FP32 instruction selection is disabled for all device code.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
OUT = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libfft3d.so")
ARCH = os.environ.get("FFT3D_ARCH", "gfx950")
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
CFLAGS = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wno-unused-command-line-argument"]


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC)
                  if f.endswith((".hip", ".cpp")))


def _compile(src):
    obj = os.path.join(OUT, os.path.basename(src) + ".o")
    cmd = [HIPCC] + CFLAGS + ["-c", src, "-o", obj]
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s" % (src, r.stdout))
    return obj


def build(jobs: int | None = None, verbose: bool = True) -> str:
    """Compile every source and link libfft3d.so; returns the library path."""
    os.makedirs(OUT, exist_ok=True)
    srcs = sources()
    jobs = jobs or min(len(srcs), max(1, min(8, os.cpu_count() or 1)))
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC"] + objs + ["-o", tmp]
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s" % r.stdout)
    os.replace(tmp, LIB)
    if verbose:
        print("built %s from %d sources" % (LIB, len(srcs)), file=sys.stderr)
    return LIB


# Sources whose host code holds the argument checks, planning, tuner-cache
# parsing and the no-allocation entry point's bookkeeping.
HOST_LOGIC = ("fft3d_api.cpp", "fft3d_many.cpp", "fft3d_noalloc.hip")
# AddressSanitizer and UndefinedBehaviorSanitizer for the host pass only:
# every -fsanitize= goes right after -Xarch_host (device code is unchanged).
HOST_SANITIZE = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                 "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]


def build_host_sanitized(out_dir: str) -> str:
    """libfft3d.so with the host code of HOST_LOGIC instrumented by ASan and
    UBSan (the other objects as build() makes them); returns its path.  Load
    it with the compiler's ASan runtime preloaded."""
    os.makedirs(out_dir, exist_ok=True)
    srcs = sources()
    plain = [s for s in srcs if os.path.basename(s) not in HOST_LOGIC]
    objs = []
    for src in plain:
        obj = os.path.join(OUT, os.path.basename(src) + ".o")
        if not os.path.exists(obj) or os.path.getmtime(obj) < os.path.getmtime(src):
            os.makedirs(OUT, exist_ok=True)
            _compile(src)
        objs.append(obj)

    def san(src):
        obj = os.path.join(out_dir, os.path.basename(src) + ".san.o")
        cmd = [HIPCC] + CFLAGS + HOST_SANITIZE + ["-c", src, "-o", obj]
        r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
        if r.returncode != 0:
            raise RuntimeError("hipcc (sanitized host) failed for %s:\n%s" % (src, r.stdout))
        return obj

    with cf.ThreadPoolExecutor(max_workers=len(HOST_LOGIC)) as ex:
        objs += list(ex.map(san, [os.path.join(CSRC, f) for f in HOST_LOGIC]))
    lib = os.path.join(out_dir, "libfft3d_hostsan.so")
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-shared-libsan"] + HOST_SANITIZE[:4] + objs + [
        "-o", lib]
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError("link (sanitized host) failed:\n%s" % r.stdout)
    return lib


if __name__ == "__main__":
    build()
