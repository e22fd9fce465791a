"""Host logic of bench.py (CPU): the live roofline's arithmetic and choice of
the dominant kernel, the guard that withholds a counter-measured traffic figure
once its kernel's source has changed, and the refusal of more than one GPU."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def info(**kw):
    base = dict(spmv_ms=0.0, spmv_launches=0, spmv_bytes=0.0, price_ms=0.0, price_launches=0,
                price_elems=0.0, diag_ms=0.0, diag_launches=0, diag_flops=0.0, update_ms=0.0,
                update_launches=0, update_flops=0.0)
    base.update(kw)
    return base


def test_committed_traffic_figures_belong_to_the_committed_kernels():
    """Every counter figure in the table was taken on the kernel text now in
    the sources, so the bench reports it rather than null."""
    for (kernel, cfg), t in bench.KERNEL_TRAFFIC.items():
        assert bench.kernel_source_sha256(t["source"], t["functions"]) == t["sha256"], kernel
        assert bench.measured_traffic(kernel, cfg) == t["bytes_per_launch"]


def test_traffic_is_withheld_for_a_changed_or_unmeasured_kernel(monkeypatch):
    key = ("cg_step", "c3")
    stale = dict(bench.KERNEL_TRAFFIC[key], sha256="0" * 64)
    monkeypatch.setitem(bench.KERNEL_TRAFFIC, key, stale)
    assert bench.measured_traffic(*key) is None
    assert bench.measured_traffic("cg_step", "c1") is None
    assert bench.kernel_source_sha256("paper_2206_11009_amd/csrc/dense.hip",
                                      ["no_such_kernel"]) is None


def test_kernel_text_hash_covers_only_the_named_function(tmp_path, monkeypatch):
    src = tmp_path / "k.hip"
    src.write_text("__global__ void a(int x) {\n    x += 1;\n}\n\n"
                   "__global__ void b(int y) {\n    y += 2;\n}\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    ha = bench.kernel_source_sha256("k.hip", ["a"])
    src.write_text("__global__ void a(int x) {\n    x += 1;\n}\n\n"
                   "__global__ void b(int y) {\n    y += 3;\n}\n")
    assert bench.kernel_source_sha256("k.hip", ["a"]) == ha
    src.write_text("__global__ void a(int x) {\n    x += 5;\n}\n\n"
                   "__global__ void b(int y) {\n    y += 3;\n}\n")
    assert bench.kernel_source_sha256("k.hip", ["a"]) != ha


def test_roofline_reports_the_kernel_with_the_largest_total_time():
    # two sampled solves: the CG iteration has the largest total time
    infos = [info(spmv_ms=300.0, spmv_launches=40000, spmv_bytes=40000 * 9.7e6,
                  price_ms=5.0, price_launches=40, price_elems=40 * 2.68e8,
                  diag_ms=100.0, diag_launches=4000, diag_flops=4000 * 174762.7,
                  update_ms=20.0, update_launches=2000, update_flops=2000 * 2.45e7),
             info(spmv_ms=30.0, spmv_launches=4000, spmv_bytes=4000 * 9.7e6,
                  price_ms=4.0, price_launches=40, price_elems=40 * 2.68e8,
                  diag_ms=10.0, diag_launches=400, diag_flops=400 * 174762.7)]
    top, other, gcosts = bench.rooflines(infos, "c3")
    assert top["kernel"].startswith("CG iteration")
    assert top["launches"] == 44000
    assert top["total_ms"] == pytest.approx(330.0)
    assert top["avg_launch_us"] == pytest.approx(7.5)
    # GB/s = bytes / ms / 1e6
    assert top["achieved"] == pytest.approx(44000 * 9.7e6 / 330.0 / 1e6)
    assert top["frac"] == pytest.approx(top["achieved"] / bench.HBM_PEAK_GBS)
    assert top["unit"] == "GB/s" and top["bound"] == "hbm"
    assert top["traffic"] == bench.measured_traffic("cg_step", "c3")
    assert set(other) == {"price_pass", "ldl_diag", "ldl_update"}
    # TFLOP/s = flops / ms / 1e9
    d = other["ldl_diag"]
    assert d["achieved"] == pytest.approx(4400 * 174762.7 / 110.0 / 1e9)
    assert d["frac"] == pytest.approx(d["achieved"] / bench.FP64_VECTOR_PEAK_TF)
    p = other["price_pass"]
    assert p["achieved"] == pytest.approx(bench.PRICE_FLOPS_PER_COST * 80 * 2.68e8 / 9.0 / 1e9)
    assert gcosts == pytest.approx(80 * 2.68e8 / 9.0 / 1e6)


def test_roofline_leaves_out_kernels_that_never_ran():
    infos = [info(spmv_ms=10.0, spmv_launches=100, spmv_bytes=1e9, price_ms=20.0,
                  price_launches=4, price_elems=1e9)]
    top, other, _ = bench.rooflines(infos, "c2")
    assert top["kernel"].startswith("price_pass")
    assert set(other) == {"cg_step"}


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "single GPU" in r.stderr
    assert r.stdout == ""
