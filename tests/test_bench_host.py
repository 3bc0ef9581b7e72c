"""bench.py on the host: it measures one GPU only and refuses --gpus N > 1
(before touching any GPU), and its cost-model helpers need no GPU."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""


def test_tangent_flop_count_formula():
    sys.path.insert(0, ROOT)
    import bench
    # Q2 (matrix cores): 2 kd ne + 150 nq^3 + 6 kd ne + 2 kd (256 + 176 + 121), kd = 3 nq^3
    kd, ne = 3 * 27, 27
    assert bench.tangent_flops_per_element(2, 3) == 2 * kd * ne + 150 * 27 + 6 * kd * ne + 2 * kd * 553
    # Q3 (sum factorisation), nq = 5
    d1, nq = 4, 5
    assert bench.tangent_flops_per_element(3, 5) == (12 * nq ** 3 * d1 ** 3 + 150 * nq ** 3
                                                     + 27 * (nq ** 3 * d1 ** 2 + nq ** 2 * d1 ** 4)
                                                     + 12 * nq * d1 ** 6)


def test_cpu_baseline_sample_is_scaled_to_a_full_apply():
    """The oracle leg times whole chunks of elements and scales to one full
    apply: on the 4^3 Q2 workload with a zero budget it takes one chunk."""
    sys.path.insert(0, ROOT)
    import bench
    from workloads import WORKLOADS, make_inputs
    w = WORKLOADS["c1"]
    r = bench.cpu_baseline(w, make_inputs(w), budget_s=0.0, chunk=16)
    assert r["kind"] == "oracle" and r["unit"] == "GDOF/s" and r["value"] > 0 and r["cores"] >= 1
    assert "over 16 of the 64 elements" in r["sample"]
