"""The benchmark's command line on the CPU: it runs on exactly one GPU and
says so, before touching a device, when asked for more."""
import glob
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=60)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_committed_profiles_match_sources_and_default_configuration():
    """The committed HBM-traffic summary was taken on the current kernel
    sources and on the benchmark's default configuration, so a default run
    reports measured bytes beside its achieved rate; and the committed bench
    line is a default run of the headline workload that meets p99 1e-4."""
    sys.path.insert(0, ROOT)
    import bench

    old = sys.argv
    sys.argv = ["bench.py"]
    try:
        a = bench.parse()
    finally:
        sys.argv = old
    cfg = {"n": 1 << 24, "criterion": a.criterion, "eps": a.eps, "theta": a.theta, "precision": a.precision,
           "variant": a.variant}
    lines = sorted(glob.glob(os.path.join(ROOT, "profiles", "bench_*.json")))
    assert len(lines) == 1, lines
    line = json.load(open(lines[0]))
    c = line["config"]
    # the summary holds for the step as the line cut it into launches
    launches = {"walk": c["counts"]["walk_pass_launches"], "far": c["counts"]["far_launches"],
                "near": c["counts"]["near_launches"]}
    for kernel in ("walk", "far", "near"):
        assert bench.traffic(kernel, cfg, a.workload, launches[kernel]) is not None, kernel
        assert bench.counters(kernel, cfg, a.workload, launches[kernel]) is not None, kernel
        # a step cut into other launches (a batched walk) has other bytes per launch
        assert bench.traffic(kernel, cfg, a.workload, launches[kernel] + 1) is None, kernel
        assert bench.counters(kernel, cfg, a.workload, launches[kernel] + 1) is None, kernel
        assert bench.traffic(kernel, dict(cfg, eps=2 * cfg["eps"]), a.workload, launches[kernel]) is None
    assert all(v["traffic"] is not None for v in line["roofline"]["others"].values())
    assert c["workload"] == a.workload and c["eps"] == a.eps and c["criterion"] == a.criterion
    assert line["steps"] == a.steps and line["warmup"] == a.warmup
    assert c["p99_rel_force_error"] <= 1e-4 and c["error_sample"] == a.error_sample
    assert line["roofline"]["traffic"] is not None and line["cpu_baseline"]["kind"] == "oracle"
