"""bench.py's contract pieces that need no GPU: the one-GPU guard, the
per-transform roofline arithmetic and the counter-summary lookup."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr and r.stdout == ""


def test_transform_roofline_arithmetic():
    # one transform of 32 grids of 128^3: 16 B per point, 0.36 ms over its two kernels
    alg = 16.0 * 128 ** 3 * 32
    r = bench.transform_roofline(alg, 0.36, "k", traffic=2.0 * alg, launches=2)
    assert abs(r["achieved"] - alg / 0.36e-3 / 1e9) < 0.1
    assert abs(r["frac"] - alg / 0.36e-3 / 1e9 / 8000.0) < 1e-4
    assert r["traffic_ratio"] == 2.0 and r["unit"] == "GB/s" and r["peak"] == 8000.0 and r["launches"] == 2
    assert bench.transform_roofline(alg, 0.36, "k")["traffic_ratio"] is None


def test_traffic_lookup_requires_current_sources(tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    units = bench.kernel_units(["k_axis_str<128, 1, 64, false, 0>"])
    h = bench.source_hash(units)
    d = {"source_hash": h, "units": units,
         "kernels": {"k_axis_str<128, 1, 64, false, 0>": {"hbm_bytes_per_launch": 123.0}}}
    (prof / "traffic_w.json").write_text(json.dumps(d))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("w", "k_axis_str<128, 1") == 123.0          # a prefix of the name
    assert bench.traffic_sum("w", ["k_axis_str<128, 1", "k_missing<"]) is None
    d["source_hash"] = "other"
    (prof / "traffic_w.json").write_text(json.dumps(d))
    assert bench.measured_traffic("w", "k_axis_str<128, 1") is None            # taken on other kernel code


def test_unit_hash_follows_the_kernels_sources():
    """A summary's hash covers the translation units of its kernels and what
    they include (the kernels' headers, the host planning code), and no
    other kernel family's sources."""
    fp32 = bench.kernel_units(["k_plane_pf<128, 1, false, true, 0>", "k_axis_str<128, 1, 64, false, 0, 0>"])
    closure = bench._include_closure(fp32)
    assert "kernels_fp32.hpp" in closure and "engine.hpp" in closure and "fft3d_api.cpp" in closure
    assert "kernels_q16.hpp" not in closure and "k_q16.hip" not in closure
    q16 = bench._include_closure(bench.kernel_units(["k_q16_plane<128, 1, 1, false, true>"]))
    assert "kernels_q16.hpp" in q16
    with pytest.raises(KeyError):
        bench.kernel_units(["k_unknown<1>"])
