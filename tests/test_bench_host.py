"""Host-side logic of bench.py (no GPU): the algorithmic byte counts behind
the roofline, the HBM-traffic table and its copy calibration, and the
one-GPU contract.
"""
import importlib.util
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_under_test",
                                                  os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_algorithmic_bytes_per_fine_node(bench):
    # FP64: read u and b, write the new iterate (24 B) and one coarse value
    # per 2^d fine nodes (the coarse right-hand side or the correction); the
    # chained 2D kernel reads u1, b, e_c and writes u, the next u1 and b_c
    assert bench.sweep_bytes_per_pt("smooth_restrict", 2) == 26.0
    assert bench.sweep_bytes_per_pt("smooth_restrict", 3) == 25.0
    assert bench.sweep_bytes_per_pt("smooth_correct", 2) == 26.0
    assert bench.sweep_bytes_per_pt("smooth_correct", 3) == 25.0
    assert bench.sweep_bytes_per_pt("post_pre_restrict", 2) == 36.0
    for kind in bench.SWEEP_KINDS:
        for d in (2, 3):
            assert bench.level_bytes_per_pt(kind, d) == bench.sweep_bytes_per_pt(kind, d)
    # the zero-guess sweeps read no iterate
    assert bench.level_bytes_per_pt("smooth_zero", 3) == 16.0
    assert bench.level_bytes_per_pt("zero_smooth_restrict", 2) == 18.0
    assert bench.level_bytes_per_pt("tail", 2) is None


def test_counter_table_is_consistent_with_the_algorithmic_bytes(bench):
    # the copy calibration: FETCH_SIZE counts half the copied bytes,
    # WRITE_SIZE all of them; every measured kernel moves at least its
    # algorithmic bytes and at most 15% more (halo re-reads)
    for name, (cbytes, cfetch, cwrite) in bench.PMC_COPY.items():
        assert cbytes / (cfetch * 1024.0) == pytest.approx(2.0, rel=1e-3)
        assert cbytes / (cwrite * 1024.0) == pytest.approx(1.0, rel=1e-3)
    for (name, kind) in bench.PMC:
        if ":" in name:
            # refinement sweeps at 3D N=512: the FP32 fused pre-smoother
            # re-reads its ring-3 halo from HBM (1.35x)
            sb = bench.STORAGE_BYTES[name.split(":")[1]]
            algo = bench.lowprec_bytes_per_pt(kind, sb) * 511 ** 3
            hi = 1.4
        else:
            d, N = bench.WORKLOADS[name]
            algo = bench.sweep_bytes_per_pt(kind, d) * (N - 1) ** d
            hi = 1.15
        ratio = bench.hbm_traffic(name, kind) / algo
        assert 1.0 <= ratio <= hi, (name, kind, ratio)
    assert bench.hbm_traffic("poisson2d_n4096", "no_such_kernel") is None


def test_more_than_one_gpu_is_refused():
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120)
    assert out.returncode == 2
    assert "one GPU only" in out.stdout


def test_closed_form_sine_solution_solves_the_sine_part(bench):
    # the bench's error reference for the mixed-precision workload: A_h of the
    # closed-form solution reproduces the sine-mode right-hand side (the
    # oracle's residual, relative to b, at rounding level)
    import oracle as O
    from paper_2206_05543_amd.workloads import poisson_problem, sine_sum
    N = 32
    p = poisson_problem(3, N, seed=3, n_modes=16, kmax=12)
    u = bench.closed_form_sine_solution(N, p["modes"], p["weights"], "cpu").numpy()
    b = sine_sum(3, N, p["modes"], p["weights"])
    r = O.residual(3, N, u, b)
    assert np.linalg.norm(r) <= 1e-12 * np.linalg.norm(b)


def test_host_cpu_fields(bench):
    h = bench.host_cpu()
    assert h["nproc"] >= 1 and 1 <= h["affinity"] <= h["nproc"]


def test_adjoint_bytes_per_fine_node(bench):
    # forward recomputation 2 x (32 + c), reverse 2 x 40 + (8 + c) + (32 + c);
    # an FP32 checkpoint is read as stored: 4 bytes of u instead of 8
    assert bench.adjoint_bytes_per_pt(2) == 64 + 4 + 80 + 40 + 4
    assert bench.adjoint_bytes_per_pt(3) == 64 + 2 + 80 + 40 + 2
    assert bench.adjoint_bytes_per_pt(3, "fp32") == bench.adjoint_bytes_per_pt(3) - 4


def test_lowprec_bytes_and_roofline(bench):
    # FP16 storage: 3 x 2 B + 2/8 B for the two smoothing sweeps, 2 x 2 B +
    # 2/8 B for the zero-guess one, 24 + 2 x 2 B for the FP64 step
    assert bench.lowprec_bytes_per_pt("smooth_restrict", 2) == 6.25
    assert bench.lowprec_bytes_per_pt("smooth_correct", 4) == 12.5
    assert bench.lowprec_bytes_per_pt("zero_smooth_restrict", 2) == 4.25
    assert bench.lowprec_bytes_per_pt("ir_step", 2) == 28.0
    rows = {"smooth_restrict": {"kernel": "a", "launches_per_solve": 6, "avg_us": 380.0,
                                "bytes_per_pt": 6.25, "GBps": 2000.0, "frac_of_peak": 0.25},
            "smooth_correct": {"kernel": "b", "launches_per_solve": 12, "avg_us": 310.0,
                               "bytes_per_pt": 6.25, "GBps": 2600.0, "frac_of_peak": 0.325},
            "ir_step": {"kernel": "c", "launches_per_solve": 7, "avg_us": 820.0,
                        "bytes_per_pt": 28.0, "GBps": 4500.0, "frac_of_peak": 0.56}}
    r = bench.lowprec_roofline({"fp16_ir": {"fine_kernels": rows}})
    # the storage-precision sweep with the most time per solve (12 x 310 us)
    assert r["frac"] == 0.325 and r["avg_launch_us"] == 310.0
    assert r["algorithmic_bytes_per_launch"] == 6.25 * 511 ** 3
    assert bench.lowprec_roofline({}) is None
