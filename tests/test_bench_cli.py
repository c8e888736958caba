"""bench.py's command-line contract that needs no GPU."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert p.returncode == 2
    msg = json.loads(p.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_kernel_hash_is_stable():
    sys.path.insert(0, ROOT)
    import bench
    assert bench.kernel_hash() == bench.kernel_hash()
    assert len(bench.kernel_hash()) == 16


def test_counter_figures_are_used_only_for_the_sources_they_were_taken_on():
    """Traffic and the FP64 VALU rate come from committed counter runs keyed
    by a hash of the kernel sources: any other hash or batch size gives
    None, never a stale figure."""
    sys.path.insert(0, ROOT)
    import bench
    n = 1 << 26
    rec = json.load(open(bench.PMC_FILE))["spd_fe_64m_f64_soa"]
    h = rec["kernel_hash"]
    assert bench.pmc_traffic(n, "0" * 16) is None
    assert bench.fp64_valu_rate(n, "0" * 16, 1.6) is None
    assert bench.pmc_traffic(n + 1, h) is None
    assert bench.pmc_traffic(n, h) == rec["hbm_bytes_per_launch"]
    r = bench.fp64_valu_rate(n, h, 2.0)
    assert r["peak"] == 78.6 and r["unit"] == "TFLOP/s"
    assert abs(r["achieved"] - rec["fp64_lane_flops_per_launch"] / 2e-3 / 1e12) < 1e-9
    assert 0 < r["frac"] < 1
