#!/usr/bin/env python3
"""Throughput of the complex 3D FFT hot path on one MI355X.

One step = the inverse transform (G -> r) followed by the forward transform
(r -> G) of a batch of sphere-cutoff plane-wave grids, both through
libfft3d's C ABI, inputs resident in HBM.  Default workload: 32 grids of
128^3 complex64 (the large FP32 batch).

Prints ONE JSON line.  `value` is nominal GFLOP/s, 5 N^3 log2(N^3) per
transform; the roofline object describes the dominant kernel (HBM-bound:
algorithmic bytes = one read of the input + one write of the output per
launch, 16 B per point); `cpu_baseline` times the FP64 oracle on the host.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X published HBM3E bandwidth

WORKLOADS = {
    # name: (n, batch, seed0, description)
    "batch128": (128, 32, 3000, "c2c 3D FFT, 32 grids of 128^3, inverse then forward, complex64"),
    "single128": (128, 1, 2128, "c2c 3D FFT, one 128^3 grid, inverse then forward, complex64"),
    "single64": (64, 1, 2064, "c2c 3D FFT, one 64^3 grid, inverse then forward, complex64"),
    "batch64": (64, 256, 4000, "c2c 3D FFT, 256 grids of 64^3, inverse then forward, complex64"),
}


def source_hash() -> str:
    h = hashlib.sha1()
    csrc = os.path.join(ROOT, "paper_2006_08435_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".hpp", ".cpp")):
            with open(os.path.join(csrc, f), "rb") as fh:
                h.update(f.encode() + b"\0" + fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload: str, kernel: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None when the summary is missing or was taken on different kernel code."""
    path = os.path.join(ROOT, "profiles", "traffic_%s.json" % workload)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("source_hash") != source_hash():
        return None
    k = d.get("kernels", {}).get(kernel)
    return None if k is None else k.get("hbm_bytes_per_launch")


def make_input(n, batch, seed0):
    import numpy as np
    import workloads
    x = np.empty((batch, n, n, n), np.complex64)
    for j in range(batch):
        x[j] = workloads.sphere_grid(n, seed0 + j)
    return x


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="batch128", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of one workload buffer (for counter scaling)")
    args = ap.parse_args(argv)
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build runs on a single MI355X; "
              "run with --gpus 1", file=sys.stderr)
        return 2

    import numpy as np
    import torch
    import paper_2006_08435_amd as fft3d
    from paper_2006_08435_amd import _lib

    n, batch, seed0, desc = WORKLOADS[args.workload]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    t_gen = time.time()
    x = make_input(n, batch, seed0)
    print("[bench] input %s generated in %.1fs" % (x.shape, time.time() - t_gen), file=sys.stderr, flush=True)
    a = torch.from_numpy(x).to(dev)
    b = torch.empty_like(a)
    c = torch.empty_like(a)
    if args.copy_calibration:
        for _ in range(args.steps):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_read": a.numel() * 8, "copies": args.steps}))
        return 0
    inv = fft3d.Plan(n, n, n, batch, "fp32", fft3d.FFT3D_INVERSE)
    fwd = fft3d.Plan(n, n, n, batch, "fp32", fft3d.FFT3D_FORWARD)
    stream = torch.cuda.current_stream()
    sh = int(stream.cuda_stream)
    L = _lib.lib()

    def step():
        inv.exec_ptr(a.data_ptr(), b.data_ptr(), sh)
        fwd.exec_ptr(b.data_ptr(), c.data_ptr(), sh)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    ms_step = e0.elapsed_time(e1) / args.steps
    print("[bench] %d steps, %.4f ms/step" % (args.steps, ms_step), file=sys.stderr, flush=True)

    # Per-kernel average launch durations (HIP events on the launch stream).
    passes = []
    for name, plan, src, dst in (("inverse", inv, a, b), ("forward", fwd, b, c)):
        for k in range(L.fft3d_plan_passes(plan.handle)):
            for _ in range(3):
                _lib.check(L.fft3d_exec_pass(plan.handle, k, src.data_ptr(), dst.data_ptr(), sh))
            reps = max(10, args.steps)
            s0 = torch.cuda.Event(enable_timing=True)
            s1 = torch.cuda.Event(enable_timing=True)
            s0.record(stream)
            for _ in range(reps):
                _lib.check(L.fft3d_exec_pass(plan.handle, k, src.data_ptr(), dst.data_ptr(), sh))
            s1.record(stream)
            torch.cuda.synchronize()
            passes.append({"transform": name, "pass": k, "ms": s0.elapsed_time(s1) / reps})
    # restore b, c from a (the pass loops above overwrote them)
    step()
    torch.cuda.synchronize()

    # Accuracy of this very run against the FP64 oracle on sampled grids.
    import oracle
    sample = sorted(set([0, batch // 2, batch - 1]))
    psi = b.cpu().numpy()
    back = c.cpu().numpy()
    errs_inv, errs_rt = [], []
    for j in sample:
        ref = oracle.fft3d(x[j].astype(np.complex128), 1)
        errs_inv.append(float(np.linalg.norm(psi[j] - ref) / np.linalg.norm(ref)))
        errs_rt.append(float(np.linalg.norm(back[j] / n ** 3 - x[j]) / np.linalg.norm(x[j])))
    ref = oracle.fft3d(psi[sample[0]].astype(np.complex128), -1)
    err_fwd = float(np.linalg.norm(back[sample[0]] - ref) / np.linalg.norm(ref))

    flops_per_transform = 5.0 * n ** 3 * math.log2(n ** 3) * batch
    gflops = 2 * flops_per_transform / (ms_step * 1e-3) / 1e9
    bytes_per_transform = 16.0 * n ** 3 * batch
    hbm_gbs = 2 * bytes_per_transform / (ms_step * 1e-3) / 1e9

    # dominant kernel: largest average launch duration
    dom = max(passes, key=lambda p: p["ms"])
    kernel_list = inv.describe().split("kernels=")[1].split(",")
    dom_name = kernel_list[dom["pass"]]
    achieved = bytes_per_transform / (dom["ms"] * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": measured_traffic(args.workload, dom_name),
                "kernel": "%s<%d,%s>" % (dom_name, n, "-1" if dom["transform"] == "forward" else "1"),
                "ms_per_launch": round(dom["ms"], 5)}

    cpu = None
    if not args.no_cpu_baseline:
        threads = oracle.max_threads()
        done, t0 = 0, time.time()
        while time.time() - t0 < args.cpu_seconds:
            y = oracle.fft3d(x[done % batch].astype(np.complex128), 1)
            oracle.fft3d(y, -1)
            done += 1
        dt = time.time() - t0
        cpu = {"value": round(2 * 5.0 * n ** 3 * math.log2(n ** 3) * done / dt / 1e9, 3), "unit": "GFLOP/s",
               "cores": threads, "kind": "oracle",
               "sample": "%d grid transforms (cycling over the %d grids), inverse then forward, FP64 "
                         "recursive radix-5/3/2 FFT, %.1f s" % (done, batch, dt)}

    out = {
        "metric": "3D FFT GFLOP/s (5N^3log2N^3/t) + HBM GB/s vs plain FP32, at rel-L2 err vs FP64",
        "value": round(gflops, 1), "unit": "GFLOP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 5), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": desc, "n": n, "batch": batch, "precision": "fp32",
                   "input": "sphere-cutoff plane-wave coefficients, seeds %d+j" % seed0},
        "hbm_gbs_algorithmic": round(hbm_gbs, 1),
        "hbm_frac_algorithmic": round(hbm_gbs / HBM_PEAK_GBS, 4),
        "rel_l2_vs_fp64": {"inverse_max": max(errs_inv), "forward": err_fwd, "round_trip_max": max(errs_rt),
                           "grids": sample},
        "kernels": [{"transform": p["transform"], "pass": p["pass"], "ms": round(p["ms"], 5)} for p in passes],
        "plans": {"inverse": inv.describe(), "forward": fwd.describe()},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "source_hash": source_hash(),
    }
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
