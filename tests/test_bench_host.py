"""Host logic of bench.py (CPU only): the one-GPU contract, the kernel-rate
arithmetic of the JSON line, the validity check of the committed counter
records, and the workload descriptions."""
import hashlib
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=60)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_cycle_step_time():
    ct = [1.0, 3.0, 6.0, 10.0, 15.0]        # end of iterations 1..5
    assert bench.cycle_step_time(ct, 0, 2) == pytest.approx(1.5)    # iterations 1, 2
    assert bench.cycle_step_time(ct, 2, 3) == pytest.approx(4.0)    # iterations 3, 4, 5
    with pytest.raises(RuntimeError):
        bench.cycle_step_time(ct, 3, 3)      # the solve ended before the last timed iteration
    with pytest.raises(RuntimeError):
        bench.cycle_step_time(ct, 0, 0)


def test_kernel_rates_arithmetic():
    stats = dict(t_matvec=2.0, n_matvec_launch=4, bytes_matvec=8e9,
                 t_dots=1.0, n_dots_launch=2, bytes_dots=5e9,
                 t_update=0.0, n_update_launch=0, bytes_update=0.0,
                 t_cg=0.5, cg_iters=10, bytes_cg=2e9, cg_max_iters=3,
                 t_gemm=0.25, flops_gemm=5e12, n_gemm_launch=5,
                 t_ritz=0.1, t_resid=0.2)
    out = bench.kernel_rates(stats)
    assert out["matvec"]["gbps"] == pytest.approx(4.0)
    assert out["matvec"]["avg_us"] == pytest.approx(5e5)
    assert out["matvec"]["bytes_per_launch"] == pytest.approx(2e9)
    assert out["dots"]["gbps"] == pytest.approx(5.0)
    assert "update" not in out                      # nothing timed, nothing reported
    assert out["cg"]["avg_us_per_iter"] == pytest.approx(5e4)
    assert out["cg"]["gbps"] == pytest.approx(4.0)
    assert out["gemm"]["tflops"] == pytest.approx(20.0)
    assert out["ritz_seconds"] == 0.1 and out["resid_seconds"] == 0.2


def test_traffic_record_only_for_its_workload_and_source():
    assert bench.traffic_for("no_such_kernel", "stencil16") is None
    for kernel in ("dots", "update"):
        path = os.path.join(ROOT, "profiles", f"traffic_{kernel}.json")
        rec = json.load(open(path))
        src = os.path.join(ROOT, rec["source"])
        current = hashlib.sha256(open(src, "rb").read()).hexdigest() == rec["source_sha256"]
        got = bench.traffic_for(kernel, rec["bench_workload"])
        assert got == (rec["hbm_bytes_per_launch"] if current else None)
        other = "stencil32" if rec["bench_workload"] != "stencil32" else "stencil16"
        assert bench.traffic_for(kernel, other) is None
        # the record's scaled counters add up to its HBM bytes
        hbm = (rec["fetch_kib_per_launch"] * 1024 * rec["fetch_scale"]
               + rec["write_kib_per_launch"] * 1024 * rec["write_scale"])
        assert hbm == pytest.approx(rec["hbm_bytes_per_launch"], rel=1e-3)


@pytest.mark.parametrize("name", sorted(bench.WORKLOADS))
def test_workload_descriptions(name):
    text = bench.describe(bench.WORKLOADS[name])
    assert isinstance(text, str) and len(text) > 20


def test_default_workload_shape():
    w = bench.WORKLOADS["stencil16"]
    assert tuple(w["L"]) == (16, 16, 16, 16)
    assert (w["nev"], w["m"], w["mwin"]) == (100, 300, 150)
    assert "n=524288" in bench.describe(w)
