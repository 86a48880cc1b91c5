"""Host logic of bench.py (no GPU): the large-image roofline arithmetic, the
traffic files' source check, the kernel-byte bound, and the refusal of
more than one GPU."""

import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def fake_large(form="f32", grid_ms=700.0, degrid_ms=800.0):
    return {"form": form, "chunks": 13, "gridder_ms_per_step": grid_ms,
            "degridder_ms_per_step": degrid_ms, "sample_taps": 1.75e12, "taps": 4.35e11}


def test_large_image_roofline_arithmetic():
    r = bench.large_image_roofline(fake_large())
    t = 0.8                                   # the degridder took longer
    assert r["kernel"] == "k_degrid" and r["bound"] == "alu" and r["unit"] == "TFLOP/s"
    assert r["achieved"] == pytest.approx(8 * 1.75e12 / t / 1e12)
    assert r["peak"] == pytest.approx(157.3)
    assert r["frac"] == pytest.approx(r["achieved"] / r["peak"])
    assert r["kernel_ms_per_launch"] == pytest.approx(800.0 / 13)
    # vector-memory bytes: a kernel value and four grid values per tap
    assert r["vmem_bytes_per_launch"] == pytest.approx(4.35e11 * (8 + 4 * 8) / 13)
    assert r["vmem_bytes_per_clk_per_cu"] == pytest.approx(
        r["vmem_bytes_per_launch"] / (t / 13) / (256 * 2.4e9))
    g = bench.large_image_roofline(fake_large("f64", grid_ms=900.0))
    assert g["kernel"] == "k_grid_tile" and g["peak"] == pytest.approx(78.6)
    # the gridder keeps its grid in registers: kernel values only
    assert g["vmem_bytes_per_launch"] == pytest.approx(4.35e11 * 16 / 13)


def test_traffic_files_match_their_sources():
    """Every committed traffic file was taken on the sources as they are
    (otherwise bench.py reports traffic as null)."""
    found = 0
    for w in ("large_image", "large_image_f16cf", "wproj2048", "standard2048", "standard_chunk"):
        path = os.path.join(ROOT, "profiles", w + "_traffic.json")
        tr = json.load(open(path))
        for kernel, k in tr["kernels"].items():
            assert k["source_sha256"] == bench.kernel_source_sha(kernel), (w, kernel)
            assert bench.traffic_per_launch(w, kernel, tr["form"]) == k["hbm_bytes_per_launch"]
            assert bench.traffic_per_launch(w, kernel, "no-such-form") is None
            found += 1
    assert found >= 8


def test_traffic_is_null_once_a_source_changes(monkeypatch):
    monkeypatch.setattr(bench, "kernel_source_sha", lambda kernel: "0" * 64)
    assert bench.traffic_per_launch("large_image", "k_degrid", "f32") is None


def test_cf_read_bytes_is_capped_by_the_table():
    assert bench.cf_read_bytes("f32", {"taps": 10, "cf_table_bytes": 1000}) == 80
    assert bench.cf_read_bytes("f16cf", {"taps": 10 ** 6, "cf_table_bytes": 1000}) == 1000


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr
    assert p.stdout == ""
