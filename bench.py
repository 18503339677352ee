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
import re
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
    "big256": (256, 4, 6000, "c2c 3D FFT, 4 grids of 256^3 (three-pass form), inverse then forward, complex64"),
    "big512": (512, 1, 6100, "c2c 3D FFT, one 512^3 grid (three-pass form), inverse then forward, complex64"),
}
EXTRA_WORKLOADS = ("mixed", "energy96", "fp16_128", "bf16_128", "pruned128", "real128", "copy_sweep", "soak_mixed")


CSRC = os.path.join(ROOT, "paper_2006_08435_amd", "csrc")
# The translation units that launch each profiled kernel family, and the host
# sources that choose every launch's grid and schedule.
KERNEL_UNITS = {
    "k_plane_pf": ("k_plane.hip", "k_variants.hip"), "k_plane_pruned": ("k_plane.hip",),
    "k_axis_str": ("k_axis.hip", "k_axis_large.hip", "k_variants.hip"), "k_axis_row": ("k_axis.hip", "k_axis_large.hip"),
    "k_axis_density": ("k_axis.hip",), "k_axis_energy": ("k_axis.hip",), "k_axis_hloc": ("k_axis.hip",),
    "k_sum_partials": ("k_axis.hip",), "k_sphere_copy": ("k_axis.hip",), "k_fused_xcd": ("k_fused.hip",),
    "k_many": ("k_many.hip",), "k_plane_r2c": ("k_real.hip",), "k_plane_c2r": ("k_real.hip",),
    "k_stream_copy": ("k_copy.hip",), "k_q16_": ("k_q16.hip",),
}
HOST_UNITS = ("fft3d_api.cpp",)
# the batched form's planner (work lists, schedules, tuner) launches these too
MANY_HOST_UNITS = ("fft3d_many.cpp",)


def kernel_units(kernels):
    """Translation units of the named kernels (profiler names) plus the host
    sources that plan their launches (the batched form's planner when the
    persistent kernel is among them); raises KeyError for a kernel family not
    listed above."""
    units = set(HOST_UNITS)
    for k in kernels:
        fam = next((f for f in KERNEL_UNITS if k.startswith(f)), None)
        if fam is None:
            raise KeyError("no translation unit listed for kernel %r" % k)
        units.update(KERNEL_UNITS[fam])
        if fam == "k_many":
            units.update(MANY_HOST_UNITS)
    return sorted(units)


def _include_closure(units):
    seen, todo = set(), list(units)
    while todo:
        f = todo.pop()
        if f in seen:
            continue
        seen.add(f)
        with open(os.path.join(CSRC, f)) as fh:
            for line in fh:
                m = re.match(r'\s*#\s*include\s+"([^"]+)"', line)
                if m:
                    todo.append(os.path.normpath(os.path.relpath(os.path.join(CSRC, os.path.dirname(f), m.group(1)), CSRC)))
    return sorted(seen)


def source_hash(units=None) -> str:
    """Hash of the device-code sources: every kernel source and header, or
    (units given) those translation units and everything they include."""
    h = hashlib.sha1()
    if units is None:
        files = sorted(f for f in os.listdir(CSRC) if f.endswith((".hip", ".hpp")))
    else:
        files = _include_closure(units)
    for f in files:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(f.encode() + b"\0" + fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload: str, kernel: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None when the summary is missing or was taken on different kernel code
    (its hash covers the sources of the kernels it lists, `units`)."""
    path = os.path.join(ROOT, "profiles", "traffic_%s.json" % workload)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("source_hash") != source_hash(d.get("units")):
        return None
    ks = d.get("kernels", {})
    k = ks.get(kernel)
    if k is None:   # a prefix of the profiler's kernel name, e.g. "k_plane_pf<128, 1"
        k = next((v for name, v in sorted(ks.items()) if name.startswith(kernel)), None)
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
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="batch128", choices=sorted(WORKLOADS) + list(EXTRA_WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of one workload buffer (for counter scaling)")
    ap.add_argument("--no-forms", action="store_true",
                    help="default workload only: skip the short runs of the 16-bit, mixed and energy forms")
    args = ap.parse_args(argv)
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library runs on a single MI355X; "
              "run with --gpus 1", file=sys.stderr)
        return 2

    import numpy as np
    import torch
    import paper_2006_08435_amd as fft3d
    from paper_2006_08435_amd import _lib

    if args.workload == "copy_sweep":
        return bench_copy_sweep(args)
    if args.workload == "soak_mixed":
        return bench_soak(args)
    if args.workload == "mixed":
        return bench_mixed(args)
    if args.workload == "energy96":
        return bench_energy(args)
    if args.workload == "pruned128":
        return bench_pruned(args)
    if args.workload == "real128":
        return bench_real(args)
    if args.workload in ("fp16_128", "bf16_128"):
        return bench_q16(args, args.workload[:4])
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

    # One step as its kernel launches: the passes of the inverse (a -> b,
    # then in place on b) and of the forward (b -> c, then in place on c);
    # running them in order is exactly the two fft3d_exec calls of step().
    seq = []
    for name, plan, src, dst in (("inverse", inv, a, b), ("forward", fwd, b, c)):
        for k in range(L.fft3d_plan_passes(plan.handle)):
            seq.append((name, k, plan.handle, (src if k == 0 else dst).data_ptr(), dst.data_ptr()))
    # Timed region: K steps through fft3d_exec, HIP events on the launch
    # stream around them (after W warm-up steps).
    ms_step = _time(step, args.steps, args.warmup, stream)
    print("[bench] %d steps, %.4f ms/step" % (args.steps, ms_step), file=sys.stderr, flush=True)
    # Kernel durations: K more steps as their individual launches, with a HIP
    # event on the same stream before the first launch and after every
    # launch (the events between launches cost ~2% of the step time, so the
    # step time above is taken without them).
    launch_fns = [(lambda h=h, k=k, s_=s_, d_=d_: _lib.check(L.fft3d_exec_pass(h, k, s_, d_, sh)))
                  for _, k, h, s_, d_ in seq]
    ms_events, launch_ms = timed_launches(launch_fns, args.steps, 0, stream)

    # The same steps timed one by one; where the working set would stay in
    # the 256 MB Infinity Cache, also cold: a 512 MiB streaming copy (untimed)
    # evicts it before each step.
    timing = {"warm": step_distribution(step, args.steps, stream), "cold": None,
              "ms_per_step_with_launch_events": round(ms_events, 5)}
    if a.numel() * 8 <= 64 << 20:
        f0 = torch.empty(512 << 20, dtype=torch.uint8, device=dev)
        f1 = torch.empty_like(f0)
        timing["cold"] = step_distribution(step, args.steps, stream,
                                           flush=lambda: fft3d.stream_copy(f0, f1, stream))
        del f0, f1
    passes = [{"transform": name, "pass": k, "ms": ms} for (name, k, _, _, _), ms in zip(seq, launch_ms)]
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

    # Roofline unit: one transform (one read of its input, one write of its
    # output, 16 B per point), over the summed average durations of its
    # kernels; the slower of the two transforms is reported.
    kernel_names = {name: plan.describe().split("kernels=")[1].split(",")
                    for name, plan in (("inverse", inv), ("forward", fwd))}
    sgn = {"inverse": "1", "forward": "-1"}
    per_transform = {}
    for p_ in passes:
        per_transform.setdefault(p_["transform"], []).append(p_)
    slow = max(per_transform, key=lambda t: sum(p_["ms"] for p_ in per_transform[t]))
    t_ms = sum(p_["ms"] for p_ in per_transform[slow])
    kerns = ["%s<%d, %s" % (kernel_names[slow][p_["pass"]], n, sgn[slow]) for p_ in per_transform[slow]]
    dom = max(passes, key=lambda p_: p_["ms"])
    roofline = transform_roofline(
        bytes_per_transform, t_ms, "%s transform: %s" % (slow, " + ".join("%s>" % k for k in kerns)),
        traffic_sum(args.workload, kerns), launches=len(kerns),
        dominant_pass={"kernel": "%s<%d,%s>" % (kernel_names[dom["transform"]][dom["pass"]], n,
                                                sgn[dom["transform"]]),
                       "ms": round(dom["ms"], 5),
                       "gbs_own_bytes": round(bytes_per_transform / (dom["ms"] * 1e-3) / 1e9, 1)})

    # the other forms run now, while the GPU is warm (after the CPU baseline's
    # seconds of host work, short timed loops of 30 steps measured up to 9%
    # slow)
    forms = None
    if args.workload == "batch128" and not args.no_forms:
        del a, b, c
        torch.cuda.empty_cache()
        forms = measure_forms(args)

    cpu = None
    if not args.no_cpu_baseline:
        threads = oracle.max_threads()
        done, t0 = 0, time.time()
        while time.time() - t0 < args.cpu_seconds:
            y = oracle.fft3d(x[done % batch].astype(np.complex128), 1)
            oracle.fft3d(y, -1)
            done += 1
        dt = time.time() - t0
        # the same on one core, over a quarter of the time
        oracle.set_threads(1)
        done1, t1 = 0, time.time()
        while time.time() - t1 < args.cpu_seconds / 4:
            y = oracle.fft3d(x[done1 % batch].astype(np.complex128), 1)
            oracle.fft3d(y, -1)
            done1 += 1
        dt1 = time.time() - t1
        oracle.set_threads(threads)
        cpu = {"value": round(2 * 5.0 * n ** 3 * math.log2(n ** 3) * done / dt / 1e9, 3), "unit": "GFLOP/s",
               "cores": threads, "kind": "oracle",
               "sample": "%d grid transforms (cycling over the %d grids), inverse then forward, FP64 "
                         "recursive radix-5/3/2 FFT, %.1f s" % (done, batch, dt),
               "one_core_value": round(2 * 5.0 * n ** 3 * math.log2(n ** 3) * done1 / dt1 / 1e9, 3),
               "one_core_sample": "%d grid transforms on 1 thread, %.1f s" % (done1, dt1),
               "cpu_model": cpu_model(), "host_cpu_count": os.cpu_count()}

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
        "timing": timing,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "source_hash": source_hash(),
    }
    out = with_copy_peak(out)
    if forms is not None:
        out["forms"] = forms
    print(json.dumps(out))
    return 0


def measure_forms(args):
    """Runs of the other forms' workloads with the default run's steps and
    warm-up, so that one default bench run measures them too: each as its
    own --workload would,
    its summary kept (step time, GFLOP/s, roofline fraction, rel-L2 against
    FP64 and the form's comparison figures); a failure is recorded, not
    raised."""
    import contextlib
    import io
    import torch
    runs = (("fp16_128", lambda a: bench_q16(a, "fp16")), ("bf16_128", lambda a: bench_q16(a, "bf16")),
            ("mixed", bench_mixed), ("energy96", bench_energy))
    keep = ("speedup_vs_fp32", "radix16_engine_ms", "compare_ms", "times_ms", "plans")
    forms = {}
    for name, fn in runs:
        sub = argparse.Namespace(**vars(args))
        sub.workload, sub.no_cpu_baseline = name, True   # the run's own steps and warm-up
        buf = io.StringIO()
        t0 = time.time()
        try:
            with contextlib.redirect_stdout(buf):
                fn(sub)
            rec = json.loads(buf.getvalue().strip().splitlines()[-1])
            r = rec.get("roofline") or {}
            forms[name] = dict({"workload": rec["config"]["workload"], "ms_per_step": rec["ms_per_step"],
                                "value": rec["value"], "unit": rec["unit"], "steps": sub.steps,
                                "roofline_frac": r.get("frac"), "traffic_ratio": r.get("traffic_ratio"),
                                "rel_l2_vs_fp64": rec.get("rel_l2_vs_fp64")},
                               **{k: rec[k] for k in keep if k in rec and k != "plans"})
            if name == "mixed":
                forms[name]["plan"] = rec["plans"]["many_tuned"]
        except Exception as e:   # recorded in the line, the headline stays
            forms[name] = {"error": "%s: %s" % (type(e).__name__, str(e)[:300])}
        forms[name]["wall_s"] = round(time.time() - t0, 1)
        print("[bench] form %s done in %.1fs" % (name, time.time() - t0), file=sys.stderr, flush=True)
        torch.cuda.empty_cache()
    return forms


def cpu_model():
    """The host CPU's model name (first /proc/cpuinfo entry), or None."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def _events():
    import torch
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def _time(fn, steps, warmup, stream):
    """Average ms of fn() over `steps` calls, HIP events on `stream`."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0, e1 = _events()
    e0.record(stream)
    for _ in range(steps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def timed_launches(seq, steps, warmup, stream):
    """Time `steps` repetitions of a launch sequence (a list of callables,
    each enqueueing one kernel) with a HIP event on `stream` before the
    first launch and after every launch.  Returns (ms per repetition,
    [average ms of each launch])."""
    import torch
    for _ in range(warmup):
        for f in seq:
            f()
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(len(seq) + 1)] for _ in range(steps)]
    for e in evs:
        e[0].record(stream)
        for i, f in enumerate(seq):
            f()
            e[i + 1].record(stream)
    torch.cuda.synchronize()
    total = evs[0][0].elapsed_time(evs[-1][-1]) / steps
    return total, [sum(e[i].elapsed_time(e[i + 1]) for e in evs) / steps for i in range(len(seq))]


def transform_roofline(alg_bytes, ms, kernel, traffic=None, **extra):
    """HBM roofline of one transform: its algorithmic bytes (one read of the
    input, one write of the output) over the summed average durations of
    its kernels, against 8 TB/s; traffic = counter-measured HBM bytes of the
    same kernels, traffic_ratio = traffic / algorithmic bytes."""
    achieved = alg_bytes / (ms * 1e-3) / 1e9
    r = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
         "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
         "traffic_ratio": None if traffic is None else round(traffic / alg_bytes, 3),
         "kernel": kernel, "algorithmic_bytes": alg_bytes, "ms_per_launch": round(ms, 5)}
    r.update(extra)
    return r


def traffic_sum(workload, kernels):
    t = [measured_traffic(workload, k) for k in kernels]
    return None if any(v is None for v in t) else sum(t)


def copy_peak_gbs(nbytes, reps=20):
    """Practical HBM ceiling: GB/s (read + write) of the library's streaming
    copy (fft3d_stream_copy) of an nbytes buffer into another."""
    import torch
    import paper_2006_08435_amd as fft3d
    n = max(16, nbytes // 16 * 16)
    src = torch.empty(n, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    stream = torch.cuda.current_stream()
    ms = _time(lambda: fft3d.stream_copy(src, dst, stream), reps, 3, stream)
    del src, dst
    return 2 * n / (ms * 1e-3) / 1e9


def with_copy_peak(rec):
    """Add to an HBM roofline the measured copy ceiling for the same bytes as
    one launch of its kernel (half of them read, half written), and the
    kernel's fraction of it."""
    r = rec.get("roofline") or {}
    ms = r.get("ms_per_launch") or r.get("ms_per_exec")
    if r.get("bound") == "hbm" and ms:
        gbs = copy_peak_gbs(int(r["achieved"] * 1e9 * ms * 1e-3 / 2))
        r["copy_peak"] = round(gbs, 1)
        r["frac_of_copy_peak"] = round(r["achieved"] / gbs, 4)
    return rec


def step_distribution(step, steps, stream, flush=None):
    """Per-step device times (HIP events around each step only): mean,
    median and min in ms.  flush, if given, runs untimed before each step."""
    import torch
    ev = []
    for _ in range(steps):
        if flush is not None:
            flush()
        e0, e1 = _events()
        e0.record(stream)
        step()
        e1.record(stream)
        ev.append((e0, e1))
    torch.cuda.synchronize()
    ts = sorted(a.elapsed_time(b) for a, b in ev)
    return {"mean_ms": round(sum(ts) / len(ts), 5), "median_ms": round(ts[len(ts) // 2], 5),
            "min_ms": round(ts[0], 5)}


def _base_record(metric_value, unit, args, ms, desc, config, dtype="f32"):
    return {"metric": "3D FFT GFLOP/s (5N^3log2N^3/t) + HBM GB/s vs plain FP32, at rel-L2 err vs FP64",
            "value": round(metric_value, 1), "unit": unit, "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": round(ms, 5), "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": dtype, "data": "synthetic", "config": dict({"workload": desc}, **config)}


def _many_kernels(desc):
    """Kernels a heterogeneous plan runs, from its description."""
    if "mode=persistent" in desc:
        return "k_many<1,%s>" % desc.split("threads=")[1].split()[0]
    if "mode=hybrid" in desc:
        return "hybrid: k_plane_pf + k_axis_str for %s, k_many<1,%s> for the other groups" % (
            desc.split("grouped=")[1].split()[0], desc.split("threads=")[1].split()[0])
    return "grouped: k_plane_pf + k_axis_str per group"


def bench_copy_sweep(args):
    """Device-to-device copy rate (read + write bytes per second) against the
    buffer size, for the library's streaming copy (non-temporal 16-byte
    loads and stores) and for torch's copy kernel (default cache policy).
    Source plus destination below the 256 MB Infinity Cache are served from
    it after the first repetition; above it every byte goes to HBM.  This is
    the indirect evidence of the cache's bandwidth: no counter of it is
    exposed on gfx950."""
    import torch
    import paper_2006_08435_amd as fft3d
    stream = torch.cuda.current_stream()
    rows = []
    for mib in (8, 16, 32, 64, 128, 256, 512, 1024):
        src = torch.empty(mib << 20, dtype=torch.uint8, device="cuda")
        src.fill_(1)
        dst = torch.empty_like(src)
        reps = max(20, min(400, (4096 // mib)))
        ms_nt = _time(lambda: fft3d.stream_copy(src, dst, stream), reps, 5, stream)
        ms_tc = _time(lambda: dst.copy_(src), reps, 5, stream)
        rows.append({"mib_each": mib, "src_plus_dst_mib": 2 * mib, "reps": reps,
                     "stream_copy_gbs": round(2 * (mib << 20) / (ms_nt * 1e-3) / 1e9, 1),
                     "torch_copy_gbs": round(2 * (mib << 20) / (ms_tc * 1e-3) / 1e9, 1)})
        del src, dst
        print("[bench] copy %d MiB done" % mib, file=sys.stderr, flush=True)
    best = max(r["stream_copy_gbs"] for r in rows)
    rec = _base_record(best, "GB/s", args, 0.0, "device copy rate against buffer size",
                       {"sizes_mib": [r["mib_each"] for r in rows]}, dtype="bytes")
    rec.update({"metric": "device-to-device copy GB/s (read + write)", "rows": rows,
                "roofline": None, "cpu_baseline": None})
    print(json.dumps(rec))
    return 0


def bench_soak(args):
    """Bounded soak of the persistent kernel's cross-workgroup hand-off: the
    mixed batch (256 x 64^3 + 48^3, 72^3, 96^3, 100^3, 120^3, inverse) run
    back to back --steps times in each schedule that uses the persistent
    kernel (all groups in it, and the hybrid split), every result compared
    bit for bit with that schedule's first result on the device; stops at
    the first mismatch.  fft3d_plan_check afterwards must report no expired
    bounded wait."""
    import numpy as np
    import torch
    import oracle
    import paper_2006_08435_amd as fft3d
    from paper_2006_08435_amd import _lib
    import workloads
    groups = [(64, 256)] + [(n, 1) for n in workloads.MIXED_SIZES]
    xs = [np.stack([workloads.sphere_grid(64, workloads.SEED_BATCH64 + j) for j in range(256)])]
    xs += [workloads.sphere_grid(n, workloads.SEED_MIXED + n)[None] for n in workloads.MIXED_SIZES]
    ins = [torch.from_numpy(x).cuda() for x in xs]
    outs = [torch.empty_like(t) for t in ins]
    stream = torch.cuda.current_stream()
    sh = int(stream.cuda_stream)
    iptr, optr = [t.data_ptr() for t in ins], [t.data_ptr() for t in outs]
    L = _lib.lib()
    runs = []
    t_start = time.time()
    for threads, chunk in ((1024, 1), (1024, 2), (-1024, 2)):   # the default schedule first
        plan = fft3d.PlanMany(groups, fft3d.FFT3D_INVERSE)
        plan.set_schedule(threads, chunk)
        plan.exec_ptrs(iptr, optr, sh)
        torch.cuda.synchronize()
        ref = [o.clone() for o in outs]
        worst = 0.0
        for (n, b), x, y in zip(groups, xs, ref):
            j = b - 1
            r = oracle.fft3d(x[j].astype(np.complex128), 1)
            worst = max(worst, float(np.linalg.norm(y[j].cpu().numpy() - r) / np.linalg.norm(r)))
        done, mismatch = 0, None
        for k in range(args.steps):
            for o in outs:
                o.zero_()
            plan.exec_ptrs(iptr, optr, sh)
            same = all(torch.equal(a, b) for a, b in zip(ref, outs))
            done += 1
            if not same:
                mismatch = k
                break
            if (k + 1) % 250 == 0:
                print("[bench] soak threads=%d chunk=%d: %d execs identical" % (threads, chunk, k + 1),
                      file=sys.stderr, flush=True)
        check = L.fft3d_plan_check(plan.handle)
        runs.append({"schedule": plan.describe(), "execs": done, "first_mismatch": mismatch,
                     "plan_check": check, "plan_check_text": L.fft3d_strerror(check).decode(),
                     "first_result_rel_l2_vs_fp64_max": worst})
        if mismatch is not None or check != 0:
            break
    rec = _base_record(0.0, "execs", args, 0.0, "soak of the persistent hand-off, mixed batch 256 x 64^3 + "
                       "48^3, 72^3, 96^3, 100^3, 120^3, inverse", {"groups": groups}, dtype="f32")
    rec.update({"metric": "persistent-kernel soak: bitwise-identical back-to-back execs",
                "value": sum(r["execs"] for r in runs), "runs": runs,
                "mismatches": sum(r["first_mismatch"] is not None for r in runs),
                "timeouts": sum(r["plan_check"] != 0 for r in runs),
                "wall_s": round(time.time() - t_start, 1), "roofline": None, "cpu_baseline": None})
    print(json.dumps(rec))
    return 0 if rec["mismatches"] == 0 and rec["timeouts"] == 0 else 1


def bench_mixed(args):
    """256 x 64^3 plus one each of 48^3, 72^3, 96^3, 100^3, 120^3 (inverse):
    one persistent launch (replayed from a captured graph) against per-grid
    and per-group plain launches."""
    import numpy as np
    import torch
    import oracle
    import paper_2006_08435_amd as fft3d
    import workloads
    groups = [(64, 256)] + [(n, 1) for n in workloads.MIXED_SIZES]
    xs = [np.stack([workloads.sphere_grid(64, workloads.SEED_BATCH64 + j) for j in range(256)])]
    xs += [workloads.sphere_grid(n, workloads.SEED_MIXED + n)[None] for n in workloads.MIXED_SIZES]
    ins = [torch.from_numpy(x).cuda() for x in xs]
    outs = [torch.empty_like(t) for t in ins]
    stream = torch.cuda.current_stream()
    plan = fft3d.PlanMany(groups, fft3d.FFT3D_INVERSE)
    # a new plan takes a cached tuned schedule if the tuning cache has one:
    # force the persistent default for the first timing
    plan.set_schedule(1024, 1)
    persistent_desc = plan.describe()
    # timed once with the default persistent schedule, then tuned (which may
    # pick the grouped mode); the record's value is the tuned plan's
    sh0 = int(torch.cuda.current_stream().cuda_stream)
    iptr0, optr0 = [t.data_ptr() for t in ins], [t.data_ptr() for t in outs]
    default_ms = _time(lambda: plan.exec_ptrs(iptr0, optr0, sh0), args.steps, args.warmup,
                       torch.cuda.current_stream())
    plan.tune()
    sh = int(stream.cuda_stream)
    iptr, optr = [t.data_ptr() for t in ins], [t.data_ptr() for t in outs]
    eager_ms = _time(lambda: plan.exec_ptrs(iptr, optr, sh), args.steps, args.warmup, stream)
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(stream)
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            plan.exec_ptrs(iptr, optr, int(s.cuda_stream))
    stream.wait_stream(s)
    graph_ms = _time(g.replay, args.steps, args.warmup, stream)
    # per-grid plain launches (261 fft3d_exec calls) and per-group batched launches
    singles = {n: fft3d.Plan(n, n, n, 1, "fp32", fft3d.FFT3D_INVERSE) for n, _ in groups}
    per_grid = []
    for (n, b), i, o in zip(groups, ins, outs):
        for j in range(b):
            per_grid.append((singles[n], i.data_ptr() + j * n ** 3 * 8, o.data_ptr() + j * n ** 3 * 8))
    grid_ms = _time(lambda: [p.exec_ptr(a, b, sh) for p, a, b in per_grid], max(3, args.steps // 5), 2, stream)
    batched = [(fft3d.Plan(n, n, n, b, "fp32", fft3d.FFT3D_INVERSE), i.data_ptr(), o.data_ptr())
               for (n, b), i, o in zip(groups, ins, outs)]
    group_ms = _time(lambda: [p.exec_ptr(a, b, sh) for p, a, b in batched], args.steps, args.warmup, stream)
    # the hybrid schedule fixed (big groups plain, the rest in one persistent launch)
    hyb = fft3d.PlanMany(groups, fft3d.FFT3D_INVERSE)
    hyb.set_schedule(-1024, 2)
    hybrid_ms = _time(lambda: hyb.exec_ptrs(iptr, optr, sh), args.steps, args.warmup, stream)
    g.replay()
    torch.cuda.synchronize()
    got = [o.cpu().numpy() for o in outs]
    worst = 0.0
    for (n, b), x, y in zip(groups, xs, got):
        for j in ([0, 255] if b > 1 else [0]):
            ref = oracle.fft3d(x[j].astype(np.complex128), 1)
            worst = max(worst, float(np.linalg.norm(y[j] - ref) / np.linalg.norm(ref)))
    flops = sum(5.0 * n ** 3 * math.log2(n ** 3) * b for n, b in groups)
    bytes_ = sum(16.0 * n ** 3 * b for n, b in groups)
    rec = _base_record(flops / (graph_ms * 1e-3) / 1e9, "GFLOP/s", args, graph_ms,
                       "c2c 3D FFT inverse, 256 grids of 64^3 + one each of 48^3, 72^3, 96^3, 100^3, 120^3, one "
                       "persistent launch replayed from a HIP graph, complex64",
                       {"groups": groups, "precision": "fp32", "input": "sphere-cutoff plane-wave coefficients"})
    achieved = bytes_ / (graph_ms * 1e-3) / 1e9
    rec.update({
        "hbm_gbs_algorithmic": round(achieved, 1), "hbm_frac_algorithmic": round(achieved / HBM_PEAK_GBS, 4),
        "rel_l2_vs_fp64": {"max_over_sampled_grids": worst},
        "compare_ms": {"tuned_graph": round(graph_ms, 4), "tuned_eager": round(eager_ms, 4),
                       "persistent_default_eager": round(default_ms, 4),
                       "per_grid_plain_launches_261": round(grid_ms, 4),
                       "per_group_batched_launches_6": round(group_ms, 4),
                       "hybrid_1024x2_eager": round(hybrid_ms, 4)},
        "plans": {"many_tuned": plan.describe(), "many_default": persistent_desc, "many_hybrid": hyb.describe()},
        "roofline": transform_roofline(
            bytes_, graph_ms, _many_kernels(plan.describe()),
            measured_traffic("mixed", "k_many") if "mode=persistent" in plan.describe() else None),
        "cpu_baseline": None if args.no_cpu_baseline else _cpu_oracle(xs[0], 64, 1, args.cpu_seconds, "64^3 grids"),
        "source_hash": source_hash(),
    })
    print(json.dumps(with_copy_peak(rec)))
    return 0


def bench_energy(args):
    """128 orbitals at 96^3: E = sum V |IFFT(c)|^2 (fused) and E + gradient."""
    import numpy as np
    import torch
    import oracle
    import paper_2006_08435_amd as fft3d
    from paper_2006_08435_amd import _lib
    import workloads
    B, n = 128, 96
    c = np.stack([workloads.sphere_grid(n, workloads.SEED_ORBITALS + j) for j in range(B)])
    V = workloads.smooth_potential(n, workloads.SEED_POTENTIAL)
    ct = torch.from_numpy(c).cuda()
    Vt = torch.from_numpy(V).cuda()
    psi = torch.empty_like(ct)
    grad = torch.empty_like(ct)
    E = torch.zeros((), dtype=torch.float64, device="cuda")
    gE = torch.ones((), dtype=torch.float64, device="cuda")
    plan = fft3d.Plan(n, n, n, B, "fp32", fft3d.FFT3D_INVERSE)
    L = _lib.lib()
    stream = torch.cuda.current_stream()
    sh = int(stream.cuda_stream)

    def fwd():
        _lib.check(L.fft3d_energy_fwd(plan.handle, ct.data_ptr(), Vt.data_ptr(), psi.data_ptr(), E.data_ptr(), sh))

    def e_only():
        _lib.check(L.fft3d_energy(plan.handle, ct.data_ptr(), Vt.data_ptr(), psi.data_ptr(), E.data_ptr(), sh))

    def bwd(have_psi):
        src = psi if have_psi else ct
        _lib.check(L.fft3d_energy_bwd(plan.handle, src.data_ptr(), int(have_psi), Vt.data_ptr(), gE.data_ptr(),
                                      grad.data_ptr(), sh))

    fwd_ms = _time(fwd, args.steps, args.warmup, stream)
    both_saved = _time(lambda: (fwd(), bwd(True)), args.steps, args.warmup, stream)
    # recomputing psi in the backward: the forward needs E only
    eonly_ms = _time(e_only, args.steps, args.warmup, stream)
    both_recomp = _time(lambda: (e_only(), bwd(False)), args.steps, args.warmup, stream)
    # the operator forward(V inverse(c)) with E, dense and with the orbitals' cutoff |G| < N/4
    hout = torch.empty_like(ct)
    E2 = torch.zeros((), dtype=torch.float64, device="cuda")

    def apply(pl):
        _lib.check(L.fft3d_apply_potential(pl.handle, ct.data_ptr(), Vt.data_ptr(), hout.data_ptr(), E2.data_ptr(),
                                           0, sh))

    apply_ms = _time(lambda: apply(plan), args.steps, args.warmup, stream)
    occ = torch.full((B,), 2.0, dtype=torch.float32, device="cuda")
    rho = torch.empty((n, n, n), dtype=torch.float32, device="cuda")
    dwork = torch.empty_like(ct)
    density_ms = _time(lambda: plan.density(ct, occ, rho=rho, work=dwork, stream=stream), args.steps, args.warmup,
                       stream)
    cplan = fft3d.Plan(n, n, n, B, "fp32", fft3d.FFT3D_INVERSE)
    cplan.set_cutoff((n / 4.0) ** 2)
    apply_cut_ms = _time(lambda: apply(cplan), args.steps, args.warmup, stream)
    apply(plan)
    torch.cuda.synchronize()
    h0 = hout[0].cpu().numpy()
    E_apply = E2.item()
    apply(cplan)
    torch.cuda.synchronize()
    hc0 = hout[0].cpu().numpy()
    Hc_ref = oracle.apply_potential(c[0].astype(np.complex128), V.astype(np.float64))
    g = workloads.signed_freq(n)
    msk = (g[:, None, None] ** 2 + g[None, :, None] ** 2 + g[None, None, :] ** 2) < (n / 4.0) ** 2
    fwd()
    bwd(True)
    torch.cuda.synchronize()
    E_ref, _, g_ref = oracle.energy(c[:8].astype(np.complex128), V.astype(np.float64))
    # E over all orbitals vs oracle: sum of per-orbital chunks
    E_all = 0.0
    for k in range(0, B, 16):
        e, _, _ = oracle.energy(c[k:k + 16].astype(np.complex128), V.astype(np.float64), want_grad=False)
        E_all += e
    g8 = grad[:8].cpu().numpy()
    E_fwd_value = E.item()
    e_only()
    torch.cuda.synchronize()
    E_only_value = E.item()
    fwd()
    torch.cuda.synchronize()
    assert E.item() == E_fwd_value
    flops = 5.0 * n ** 3 * math.log2(n ** 3) * B
    rec = _base_record(2 * flops / (both_saved * 1e-3) / 1e9, "GFLOP/s", args, both_saved,
                       "plane-wave local-potential energy E = sum V|IFFT(c)|^2 and its gradient, 128 orbitals at "
                       "96^3, complex64 (forward + backward from saved psi)",
                       {"orbitals": B, "n": n, "precision": "fp32",
                        "input": "sphere-cutoff orbitals, V = 16 low-|G| cosines"})
    alg = 16.0 * n ** 3 * B
    rec.update({
        "times_ms": {"energy_fwd": round(fwd_ms, 4), "energy_only_psi_not_stored": round(eonly_ms, 4),
                     "fwd_plus_bwd_saved_psi": round(both_saved, 4),
                     "fwd_plus_bwd_recompute_psi": round(both_recomp, 4),
                     "apply_potential_with_E": round(apply_ms, 4),
                     "apply_potential_with_E_cutoff": round(apply_cut_ms, 4),
                     "density_128_orbitals": round(density_ms, 4)},
        "apply_potential": {"rel_l2_orbital0": float(np.linalg.norm(h0 - Hc_ref) / np.linalg.norm(Hc_ref)),
                            "rel_l2_orbital0_inside_sphere_cutoff":
                                float(np.linalg.norm(hc0[msk] - Hc_ref[msk]) / np.linalg.norm(Hc_ref[msk])),
                            "E_rel": abs(E_apply - E_all) / abs(E_all),
                            "algorithmic_bytes_dense": 3 * alg, "hbm_gbs_dense": round(3 * alg / (apply_ms * 1e-3) / 1e9, 1)},
        "hbm_gbs_algorithmic": round(2 * alg / (both_saved * 1e-3) / 1e9, 1),
        "rel_l2_vs_fp64": {"E_rel": abs(E.item() - E_all) / abs(E_all),
                           "grad_first8": float(np.linalg.norm(g8 - g_ref) / np.linalg.norm(g_ref)),
                           "E_only_rel": abs(E_only_value - E_all) / abs(E_all)},
        # unit: the energy forward (one read of c, one write of psi; V, 3.4 MB,
        # and the partial sums are not counted)
        "roofline": transform_roofline(alg, fwd_ms, "energy_fwd: k_plane_pf<96, 1, false, true> + "
                                       "k_axis_str<96, 1, 64, true, 0> + k_sum_partials",
                                       traffic_sum("energy96", ["k_plane_pf<96, 1, false, true",
                                                                "k_axis_str<96, 1, 64, true, 0"]),
                                       launches=3),
        "cpu_baseline": None if args.no_cpu_baseline else _cpu_oracle(c, n, 1, args.cpu_seconds, "96^3 orbitals"),
        "source_hash": source_hash(),
    })
    print(json.dumps(with_copy_peak(rec)))
    return 0


def bench_pruned(args):
    """32 x 128^3 sphere-cutoff coefficients (|G| < N/4): pruned inverse then
    pruned forward (the two transforms around a local-operator product),
    against the dense inverse and forward on the same data."""
    import numpy as np
    import torch
    import oracle
    import paper_2006_08435_amd as fft3d
    import workloads
    from paper_2006_08435_amd import _lib
    n, B = 128, 32
    r2 = (n / 4.0) ** 2
    x = workloads.sphere_batch(n, [workloads.SEED_BATCH128 + j for j in range(B)])
    xt = torch.from_numpy(x).cuda()
    psi = torch.empty_like(xt)
    back = torch.empty_like(xt)
    d_psi = torch.empty_like(xt)
    d_back = torch.empty_like(xt)
    plans = {}
    for name, d in (("inverse", fft3d.FFT3D_INVERSE), ("forward", fft3d.FFT3D_FORWARD)):
        plans["dense_" + name] = fft3d.Plan(n, n, n, B, "fp32", d)
        plans[name] = fft3d.Plan(n, n, n, B, "fp32", d)
        plans[name].set_cutoff(r2)
    stream = torch.cuda.current_stream()
    sh = int(stream.cuda_stream)
    L = _lib.lib()

    def pruned_step():
        plans["inverse"].exec_ptr(xt.data_ptr(), psi.data_ptr(), sh)
        plans["forward"].exec_ptr(psi.data_ptr(), back.data_ptr(), sh)

    def dense_step():
        plans["dense_inverse"].exec_ptr(xt.data_ptr(), d_psi.data_ptr(), sh)
        plans["dense_forward"].exec_ptr(d_psi.data_ptr(), d_back.data_ptr(), sh)

    npts = plans["inverse"].sphere_points
    packed_c = plans["inverse"].pack(xt)
    packed_back = torch.empty_like(packed_c)
    work = torch.empty_like(xt)

    def packed_step():
        _lib.check(L.fft3d_exec_packed(plans["inverse"].handle, work.data_ptr(), packed_c.data_ptr(), sh))
        _lib.check(L.fft3d_exec_packed(plans["forward"].handle, work.data_ptr(), packed_back.data_ptr(), sh))

    dense_ms = _time(dense_step, args.steps, args.warmup, stream)
    packed_ms = _time(packed_step, args.steps, args.warmup, stream)
    # the pruned step as its four launches, each bracketed by HIP events
    names, seq = [], []
    for name, src, dst in (("inverse", xt, psi), ("forward", psi, back)):
        pl = plans[name]
        for k in range(L.fft3d_plan_passes(pl.handle)):
            names.append("%s_pass%d" % (name, k))
            seq.append(lambda h=pl.handle, k=k, s_=(src if k == 0 else dst).data_ptr(), d_=dst.data_ptr():
                       _lib.check(L.fft3d_exec_pass(h, k, s_, d_, sh)))
    pruned_ms = _time(pruned_step, args.steps, args.warmup, stream)
    pruned_events_ms, per = timed_launches(seq, args.steps, 0, stream)
    times = dict(zip(names, per))
    for name, src in (("inverse", xt), ("forward", psi)):
        times["dense_" + name] = _time(lambda: plans["dense_" + name].exec_ptr(src.data_ptr(), d_back.data_ptr(),
                                                                               sh), args.steps, args.warmup, stream)
    pruned_step()
    dense_step()
    packed_step()
    torch.cuda.synchronize()
    packed_rt = float(((packed_back / n ** 3) - packed_c).abs().max() / packed_c.abs().max())
    g = workloads.signed_freq(n)
    sphere = (g[:, None, None] ** 2 + g[None, :, None] ** 2 + g[None, None, :] ** 2) < r2
    ms = torch.from_numpy(np.broadcast_to(sphere[None], x.shape).copy()).cuda()
    fdiff = float((back[ms] - d_back[ms]).abs().max() / d_back[ms].abs().max())
    equal = {"inverse_bitwise": bool(torch.equal(psi, d_psi)),
             "forward_inside_sphere_max_abs_diff_over_max": fdiff}
    worst = {"inverse": 0.0, "round_trip_inside_sphere": 0.0}
    for j in (0, B - 1):
        ref = oracle.fft3d(x[j].astype(np.complex128), 1)
        y = psi[j].cpu().numpy()
        worst["inverse"] = max(worst["inverse"], float(np.linalg.norm(y - ref) / np.linalg.norm(ref)))
        rt = back[j].cpu().numpy()[sphere] / n ** 3
        worst["round_trip_inside_sphere"] = max(worst["round_trip_inside_sphere"],
                                                float(np.linalg.norm(rt - x[j][sphere]) /
                                                      np.linalg.norm(x[j][sphere])))
    # algorithmic bytes: the inverse reads the sphere's coefficients and
    # writes the whole grid, the forward reads the whole grid and writes the
    # sphere's coefficients
    zin = (g * g) < r2
    disk = int(((g[:, None] ** 2 + g[None, :] ** 2) < r2).sum())   # x-rows (inverse) = z-lines (forward)
    nzp, nsph = int(zin.sum()), int(sphere.sum())
    alg = 8.0 * (nsph + n ** 3) * B
    # bytes the pruned passes must move at least (whole rows / lines as the
    # passes fetch them, the intermediate included)
    pass_bytes = {"inverse_pass0": 8.0 * (disk * n + nzp * n * n) * B,
                  "inverse_pass1": 8.0 * (nzp * n * n + n ** 3) * B,
                  "forward_pass0": 8.0 * (n ** 3 + disk * n) * B,
                  "forward_pass1": 8.0 * (disk * n + nsph) * B}
    flops = 2 * 5.0 * n ** 3 * math.log2(n ** 3) * B
    rec = _base_record(flops / (pruned_ms * 1e-3) / 1e9, "GFLOP/s", args, pruned_ms,
                       "pruned c2c 3D FFT, sphere-cutoff coefficients (|G| < N/4), 32 grids of 128^3: inverse then "
                       "forward, complex64; GFLOP/s counts the dense 5N^3log2N^3 per transform",
                       {"n": n, "batch": B, "cutoff_r2": r2, "precision": "fp32",
                        "input": "sphere-cutoff plane-wave coefficients"})
    kern = {"inverse": ["k_plane_pruned<128, 1, 0, false", "k_axis_str<128, 1, 64, false, 1"],
            "forward": ["k_plane_pruned<128, -1, 1, false", "k_axis_str<128, -1, 64, false, 2"]}
    t_ms = {t: times[t + "_pass0"] + times[t + "_pass1"] for t in ("inverse", "forward")}
    slow = max(t_ms, key=t_ms.get)
    rec.update({
        "times_ms": dict({"pruned_step": round(pruned_ms, 4), "dense_step": round(dense_ms, 4),
                          "speedup": round(dense_ms / pruned_ms, 3),
                          "packed_step": round(packed_ms, 4),
                          "pruned_step_with_launch_events": round(pruned_events_ms, 4)},
                         **{k: round(v, 4) for k, v in times.items()}),
        "sphere": {"nonzero_planes": nzp, "disk_lines_per_grid": disk, "sphere_points_per_grid": nsph,
                   "points_per_grid": n ** 3},
        "algorithmic_bytes": {"per_transform": alg, "dense_transform": 16.0 * n ** 3 * B,
                              "pass_minimum": pass_bytes},
        "hbm_gbs_algorithmic": round(2 * alg / (pruned_ms * 1e-3) / 1e9, 1),
        "hbm_frac_algorithmic": round(2 * alg / (pruned_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "vs_dense_plans": equal,
        "packed": {"points_per_grid": npts, "round_trip_max_abs_err_over_max": packed_rt},
        "rel_l2_vs_fp64": dict(worst, sampled=[0, B - 1]),
        "plans": {k: v.describe() for k, v in plans.items()},
        "roofline": transform_roofline(alg, t_ms[slow], "%s transform: %s" % (slow, " + ".join(
            k + ">" for k in kern[slow])), traffic_sum("pruned128", kern[slow]), launches=2),
        "cpu_baseline": None if args.no_cpu_baseline else _cpu_oracle(x, n, 1, args.cpu_seconds, "128^3 grids"),
        "source_hash": source_hash(),
    })
    print(json.dumps(with_copy_peak(rec)))
    return 0


def bench_real(args):
    """32 real grids of 128^3: r2c then c2r (the c2r consumes, and
    overwrites, the r2c's half spectrum)."""
    import numpy as np
    import torch
    import oracle
    import paper_2006_08435_amd as fft3d
    from paper_2006_08435_amd import _lib
    n, B = 128, 32
    h = n // 2 + 1
    f = np.random.default_rng(9900).uniform(-1, 1, (B, n, n, n)).astype(np.float32)
    ft = torch.from_numpy(f).cuda()
    half = torch.empty((B, n, n, h), dtype=torch.complex64, device="cuda")
    back = torch.empty_like(ft)
    fwd = fft3d.RealPlan(n, n, n, B, fft3d.FFT3D_FORWARD)
    inv = fft3d.RealPlan(n, n, n, B, fft3d.FFT3D_INVERSE)
    stream = torch.cuda.current_stream()
    sh = int(stream.cuda_stream)
    L = _lib.lib()

    def step():
        _lib.check(L.fft3d_exec(fwd.handle, ft.data_ptr(), half.data_ptr(), sh))
        _lib.check(L.fft3d_exec(inv.handle, half.data_ptr(), back.data_ptr(), sh))

    # (buffers per pass: r2c = [plane ft -> half, z in place on half];
    #  c2r = [z in place on half, plane half -> back])
    names, seq = [], []
    for name, pl, bufs in (("r2c", fwd, ((ft, half), (half, half))), ("c2r", inv, ((half, half), (half, back)))):
        for k in range(L.fft3d_plan_passes(pl.handle)):
            a_, b_ = bufs[k]
            names.append("%s_pass%d" % (name, k))
            seq.append(lambda h=pl.handle, k=k, s_=a_.data_ptr(), d_=b_.data_ptr():
                       _lib.check(L.fft3d_exec_pass(h, k, s_, d_, sh)))
    ms = _time(step, args.steps, args.warmup, stream)   # the step through fft3d_exec
    ms_events, per = timed_launches(seq, args.steps, 0, stream)
    times = dict(zip(names, per))
    # the timing loop above left `half` transformed in place: recompute and check
    _lib.check(L.fft3d_exec(fwd.handle, ft.data_ptr(), half.data_ptr(), sh))
    torch.cuda.synchronize()
    H = half.cpu().numpy()
    worst = {"r2c": 0.0, "round_trip": 0.0}
    for j in (0, B - 1):
        ref = oracle.r2c3d(f[j].astype(np.float64))
        worst["r2c"] = max(worst["r2c"], float(np.linalg.norm(H[j] - ref) / np.linalg.norm(ref)))
    _lib.check(L.fft3d_exec(inv.handle, half.data_ptr(), back.data_ptr(), sh))
    torch.cuda.synchronize()
    bk = back.cpu().numpy()
    for j in (0, B - 1):
        worst["round_trip"] = max(worst["round_trip"],
                                  float(np.linalg.norm(bk[j] / n ** 3 - f[j]) / np.linalg.norm(f[j])))
    real_b, half_b = 4.0 * n ** 3, 8.0 * n * n * h
    # algorithmic bytes of each transform: its input read once, its output
    # written once (the real grid and the half spectrum)
    alg = (real_b + half_b) * B
    flops = 2 * 2.5 * n ** 3 * math.log2(n ** 3) * B
    rec = _base_record(flops / (ms * 1e-3) / 1e9, "GFLOP/s", args, ms,
                       "real 3D FFT, 32 real grids of 128^3: r2c then c2r, float32 / complex64 half spectra; "
                       "GFLOP/s counts 2.5 N^3 log2 N^3 per real transform",
                       {"n": n, "batch": B, "precision": "fp32", "input": "uniform real grids"})
    kern = {"r2c": ["k_plane_r2c<128, -1", "k_axis_str<128, -1, 64, false, 0"],
            "c2r": ["k_axis_str<128, 1, 64, false, 0", "k_plane_c2r<128, 1"]}
    t_ms = {t: times[t + "_pass0"] + times[t + "_pass1"] for t in ("r2c", "c2r")}
    slow = max(t_ms, key=t_ms.get)
    rec.update({
        "times_ms": dict({k: round(v, 4) for k, v in times.items()}, step_with_launch_events=round(ms_events, 4)),
        "algorithmic_bytes_per_transform": alg,
        "hbm_gbs_algorithmic": round(2 * alg / (ms * 1e-3) / 1e9, 1),
        "hbm_frac_algorithmic": round(2 * alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "rel_l2_vs_fp64": dict(worst, sampled=[0, B - 1]),
        "plans": {"r2c": fwd.describe(), "c2r": inv.describe()},
        "roofline": transform_roofline(alg, t_ms[slow], "%s transform: %s" % (slow, " + ".join(
            k + ", ...>" for k in kern[slow])), traffic_sum("real128", kern[slow]), launches=2),
        "cpu_baseline": None,
        "source_hash": source_hash(),
    })
    print(json.dumps(with_copy_peak(rec)))
    return 0


def bench_q16(args, prec):
    """32 x 128^3 in scaled 16-bit storage: inverse then forward, against the
    FP32 path on the same (dequantized) data; both radix-16 engines."""
    import numpy as np
    import torch
    import oracle
    import paper_2006_08435_amd as fft3d
    from paper_2006_08435_amd import _lib
    n, B = 128, 32
    x = make_input(n, B, 3000)
    xt = torch.from_numpy(x).cuda()
    qa = fft3d.quantize(xt, prec)
    qb = torch.empty_like(qa)
    qc = torch.empty_like(qa)
    stream = torch.cuda.current_stream()
    sh = int(stream.cuda_stream)
    L = _lib.lib()

    def plans(mfma):
        # the radix-16 engine is chosen at plan time (FFT3D_Q16_MFMA=1: matrix cores)
        if mfma:
            os.environ["FFT3D_Q16_MFMA"] = "1"
        try:
            return (fft3d.Plan(n, n, n, B, prec, fft3d.FFT3D_INVERSE),
                    fft3d.Plan(n, n, n, B, prec, fft3d.FFT3D_FORWARD))
        finally:
            os.environ.pop("FFT3D_Q16_MFMA", None)

    def launches(inv, fwd):
        seq = []
        for h, src, dst in ((inv.handle, qa, qb), (fwd.handle, qb, qc)):
            for k in range(L.fft3d_plan_passes(h)):
                seq.append(lambda h=h, k=k, s_=(src if k == 0 else dst).data_ptr(), d_=dst.data_ptr():
                           _lib.check(L.fft3d_exec_pass(h, k, s_, d_, sh)))
        return seq

    fmt = oracle.FMT_FP16 if prec == "fp16" else oracle.FMT_BF16
    nb = 4 * n ** 3 * B
    dec = lambda r, j: oracle.q16_decode(r[:nb].view(np.uint16).reshape(B, n, n, n, 2)[j:j + 1],
                                          r[nb:].view(np.int8).reshape(B, n, n)[j:j + 1], fmt)

    def errors(inv, fwd):
        """rel-L2 of this engine's inverse (vs FP64 on the dequantized input
        and on the original FP32 input) and forward, sampled grids."""
        inv.exec_ptr(qa.data_ptr(), qb.data_ptr(), sh)
        fwd.exec_ptr(qb.data_ptr(), qc.data_ptr(), sh)
        torch.cuda.synchronize()
        raw = {k: v.cpu().numpy() for k, v in (("a", qa), ("b", qb), ("c", qc))}
        e_inv, e_fwd, e_orig = [], [], []
        for j in (0, 16, 31):
            xin = dec(raw["a"], j)
            psi = dec(raw["b"], j)
            ri = oracle.fft3d(xin, 1)
            e_inv.append(float(np.linalg.norm(psi - ri) / np.linalg.norm(ri)))
            ref_orig = oracle.fft3d(x[j:j + 1].astype(np.complex128), 1)
            e_orig.append(float(np.linalg.norm(psi - ref_orig) / np.linalg.norm(ref_orig)))
            rf = oracle.fft3d(psi, -1)
            e_fwd.append(float(np.linalg.norm(dec(raw["c"], j) - rf) / np.linalg.norm(rf)))
        return {"inverse_vs_dequantized_input_max": max(e_inv), "forward_max": max(e_fwd),
                "inverse_vs_original_fp32_input_max": max(e_orig), "grids": [0, 16, 31]}

    inv, fwd = plans(False)
    inv_m, fwd_m = plans(True)
    # step times through fft3d_exec, then the launches with events between them
    ms = _time(lambda: (inv.exec_ptr(qa.data_ptr(), qb.data_ptr(), sh), fwd.exec_ptr(qb.data_ptr(), qc.data_ptr(), sh)),
               args.steps, args.warmup, stream)
    ms_mfma = _time(lambda: (inv_m.exec_ptr(qa.data_ptr(), qb.data_ptr(), sh),
                             fwd_m.exec_ptr(qb.data_ptr(), qc.data_ptr(), sh)), args.steps, args.warmup, stream)
    _, per_launch = timed_launches(launches(inv, fwd), args.steps, args.warmup, stream)
    _, per_launch_m = timed_launches(launches(inv_m, fwd_m), args.steps, args.warmup, stream)
    # FP32 reference path on the dequantized input, same step
    xd = fft3d.dequantize(qa, x.shape, prec)
    b32, c32 = torch.empty_like(xd), torch.empty_like(xd)
    inv32 = fft3d.Plan(n, n, n, B, "fp32", fft3d.FFT3D_INVERSE)
    fwd32 = fft3d.Plan(n, n, n, B, "fp32", fft3d.FFT3D_FORWARD)
    ms32 = _time(lambda: (inv32.exec_ptr(xd.data_ptr(), b32.data_ptr(), sh),
                          fwd32.exec_ptr(b32.data_ptr(), c32.data_ptr(), sh)), args.steps, args.warmup, stream)
    err_m = errors(inv_m, fwd_m)
    err = errors(inv, fwd)
    flops = 5.0 * n ** 3 * math.log2(n ** 3) * B
    alg = 8.0 * n ** 3 * B + 2.0 * n * n * B
    rec = _base_record(2 * flops / (ms * 1e-3) / 1e9, "GFLOP/s", args, ms,
                       "c2c 3D FFT, 32 grids of 128^3 in scaled %s storage (per-row power-of-two exponent), inverse "
                       "then forward, radix-16 stage on the vector ALUs (default engine)" % prec,
                       {"n": n, "batch": B, "precision": prec + "_scaled",
                        "input": "sphere-cutoff plane-wave coefficients, seeds 3000+j, quantized on the GPU"},
                       dtype="f32 arithmetic, %s storage" % prec)
    f = 1 if prec == "fp16" else 2

    def roof(per, mfma):
        # the slower of the two transforms (launches 0-1 inverse, 2-3 forward)
        t = max((0, 2), key=lambda i: per[i] + per[i + 1])
        sg = "1" if t == 0 else "-1"
        kern = ["k_q16_plane<128, %s, %d, %s" % (sg, f, "true" if mfma else "false"),
                "k_q16_slab<128, %s, %d, %s" % (sg, f, "true" if mfma else "false")]
        return transform_roofline(alg, per[t] + per[t + 1],
                                  "%s transform: %s" % ("inverse" if t == 0 else "forward",
                                                        " + ".join(k + ", ...>" for k in kern)),
                                  traffic_sum(args.workload, kern), launches=2)

    rec.update({
        "hbm_gbs_algorithmic": round(2 * alg / (ms * 1e-3) / 1e9, 1),
        "hbm_frac_algorithmic": round(2 * alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "rel_l2_vs_fp64": err,
        "fp32_same_step_ms": round(ms32, 5), "speedup_vs_fp32": round(ms32 / ms, 3),
        "radix16_engine_ms": {"valu_default": round(ms, 5), "mfma": round(ms_mfma, 5)},
        "mfma_engine": {"rel_l2_vs_fp64": err_m, "kernels_ms": [round(t, 5) for t in per_launch_m],
                        "roofline": roof(per_launch_m, True)},
        "kernels_ms": [round(t, 5) for t in per_launch],
        "plans": {"inverse": inv.describe(), "inverse_mfma": inv_m.describe()},
        "roofline": roof(per_launch, False),
        "cpu_baseline": None,
        "source_hash": source_hash(),
    })
    print(json.dumps(with_copy_peak(rec)))
    return 0


def _cpu_oracle(x, n, per, seconds, what):
    """Oracle (FP64, all host threads) inverse+forward on grids of x until
    `seconds` have passed."""
    import numpy as np
    import oracle
    threads = oracle.max_threads()
    done, t0 = 0, time.time()
    while time.time() - t0 < seconds:
        y = oracle.fft3d(x[done % len(x)].astype(np.complex128), 1)
        oracle.fft3d(y, -1)
        done += 1
    dt = time.time() - t0
    return {"value": round(2 * 5.0 * n ** 3 * math.log2(n ** 3) * done / dt / 1e9, 3), "unit": "GFLOP/s",
            "cores": threads, "kind": "oracle",
            "sample": "%d %s, inverse then forward, FP64 recursive radix-5/3/2 FFT, %.1f s" % (done, what, dt)}


if __name__ == "__main__":
    sys.exit(main())
