"""Host-side checks that need no GPU: the rocprofv3 summary tool (kernel names,
the counter-to-bytes scaling), the benchmark's refusal of more than one GPU,
and the argument checks of the multigrid and diagnostics entry points."""
import csv
import ctypes
import os
import subprocess
import sys

import pytest

from paper_2107_14027_amd import binding as B
from paper_2107_14027_amd import rocprof_summary as rs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.parametrize("name,short", [
    ("void fr::(anonymous namespace)::k_fused<3, double, true, false>(double const*)", "k_fused<3,double>"),
    ("void fr::(anonymous namespace)::k_fused<3, double, true, true>(double const*)", "k_fused_stage<3,double>"),
    ("void fr::(anonymous namespace)::k_fused<3, double, true, true, false>(double const*)",
     "k_fused_stage<3,double>"),
    ("void fr::(anonymous namespace)::k_fused<6, double, true, false, false>(double const*)",
     "k_fused<6,double>"),
    ("void fr::(anonymous namespace)::k_lines<2, double, true>(double const*)", "k_lines_halo<2,double>"),
    ("void fr::(anonymous namespace)::k_lines<2, float, false>(float const*)", "k_lines<2,float>"),
    ("void fr::(anonymous namespace)::k_trace<6, float, true>(float const*)", "k_trace<6,float>"),
    ("void fr::(anonymous namespace)::k_stage<double, true, false>(double*)", "k_stage<double,true,false>"),
    ("void fr::(anonymous namespace)::k_final_sum(double const*, int, double*)", "k_final_sum"),
])
def test_kernel_names(name, short):
    assert rs.short(name) == short


def write_csv(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for r in rows:
            w.writerow(r)


def test_traffic_scaling(tmp_path):
    """A copy of N bytes that FETCH_SIZE reports as N/2 KiB-units scales every
    kernel's fetch by 2; the per-launch bytes are the mean over dispatches."""
    N = 1 << 20
    kf = "void fr::(anonymous namespace)::k_fused<2, double, true, false>(double const*)"
    fetch = [dict(Dispatch_Id=1, Kernel_Name="__amd_rocclr_copyBuffer", Counter_Name="FETCH_SIZE",
                  Counter_Value=N / 2 / 1024),
             dict(Dispatch_Id=2, Kernel_Name=kf, Counter_Name="FETCH_SIZE", Counter_Value=100.0),
             dict(Dispatch_Id=2, Kernel_Name=kf, Counter_Name="FETCH_SIZE", Counter_Value=50.0),
             dict(Dispatch_Id=3, Kernel_Name=kf, Counter_Name="FETCH_SIZE", Counter_Value=250.0)]
    write = [dict(Dispatch_Id=1, Kernel_Name="__amd_rocclr_copyBuffer", Counter_Name="WRITE_SIZE",
                  Counter_Value=N / 1024),
             dict(Dispatch_Id=2, Kernel_Name=kf, Counter_Name="WRITE_SIZE", Counter_Value=40.0),
             dict(Dispatch_Id=3, Kernel_Name=kf, Counter_Name="WRITE_SIZE", Counter_Value=60.0)]
    fp, wp = tmp_path / "f.csv", tmp_path / "w.csv"
    write_csv(fp, fetch)
    write_csv(wp, write)
    argv = sys.argv
    sys.argv = ["rocprof_summary", "traffic", str(fp), str(wp), str(tmp_path), "--calib-bytes", str(N),
                "--command-fetch", "f", "--command-write", "w"]
    try:
        rs.main()
    finally:
        sys.argv = argv
    txt = (tmp_path / "traffic_k_fused_p2_f64.txt").read_text()
    vals = dict(line.split(": ", 1) for line in txt.splitlines() if ": " in line and not line.startswith("#"))
    assert float(vals["fetch_scale"]) == pytest.approx(2.0)
    assert float(vals["write_scale"]) == pytest.approx(1.0)
    # fetch: dispatch 2 sums its entries (150), dispatch 3 is 250 -> mean 200 KiB, x2
    assert float(vals["hbm_read_bytes_per_launch"]) == pytest.approx(200 * 1024 * 2.0)
    assert float(vals["hbm_write_bytes_per_launch"]) == pytest.approx(50 * 1024 * 1.0)
    assert vals["source_sha256_16"] == rs.kernel_source_hash()


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_new_entry_points_validate_arguments():
    L = B.lib()
    assert L.fr_pmg_create(None, 0, None, None, 1.75) is None
    assert b"NULL" in L.fr_last_error()
    L.fr_pmg_destroy(None)
    it = ctypes.c_int()
    res = ctypes.c_double()
    assert L.fr_pmg_dual_step(None, None, None, None, 1e-2, 1e-3, 1e-6, 3, ctypes.byref(it),
                              ctypes.byref(res), None) == B.FR_EINVAL
    out = (ctypes.c_double * 2)()
    assert L.fr_diagnostics(None, None, out, None) == B.FR_EINVAL
    assert L.fr_acm_create(None, 0.5, 0.1) is None
    L.fr_acm_destroy(None)
    assert L.fr_acm_residual(None, None, None, None) == B.FR_EINVAL
    assert L.fr_acm_gradient(None, None, None, None) == B.FR_EINVAL
    assert L.fr_acm_dual_step(None, None, None, None, 1e-2, 1e-3, 1e-6, 3, 1, ctypes.byref(it),
                              ctypes.byref(res), None) == B.FR_EINVAL
    assert L.fr_lhex_create(None) is None
    L.fr_lhex_destroy(None)
    assert L.fr_lhex_residual(None, None, None, None, None) == B.FR_EINVAL


def test_bench_closed_form_manufactured_operator():
    """bench.py's closed form of -div F + S for P = u = v = w = sin x sin y sin z
    (the matrix-core precision study's error reference) equals the symbolic
    differentiation of the flux."""
    import numpy as np
    import bench
    from test_oracle_residual import sines_exact_residual
    for p, n in ((2, (2, 3, 2)), (4, (2, 2, 2))):
        E = sines_exact_residual(p, n)
        C = bench.sines_operator(p, n)
        assert np.max(np.abs(C - E[:, :4])) <= 1e-13
        assert np.max(np.abs(E[:, 4:])) <= 1e-13
