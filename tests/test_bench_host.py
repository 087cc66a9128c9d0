"""Host-side logic of bench.py (no GPU): workloads, algorithmic bytes, the
lookup of committed HBM-traffic summaries, and the one-GPU guard."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_2408_00146_amd import cases  # noqa: E402


def test_bytes_per_node_are_72_populations():
    # 36 loads + 36 stores per lattice update, per storage type
    assert bench.BYTES_PER_NODE == {cases.FP64: 72 * 8, cases.FP32: 72 * 4, cases.FP16S: 72 * 2}


def test_default_workload_shape():
    ps = bench.workload("fp32_1024x512x4")
    assert len(ps) == 4
    assert all(p["nx"] == 1024 and p["ny"] == 512 and p["precision"] == cases.FP32 for p in ps)
    assert sum(p["nx"] * p["ny"] for p in ps) == 2097152


@pytest.mark.parametrize("name", bench.COMPARE)
def test_compare_workloads_exist(name):
    ps = bench.workload(name)
    assert ps and all(p["nx"] > 0 and p["ny"] > 0 for p in ps)


def test_unknown_workload_is_rejected():
    with pytest.raises(SystemExit):
        bench.workload("no_such_workload")


def test_traffic_lookup_matches_committed_summary():
    """Every traffic summary under profiles/ is found for its own workload and
    kernel configuration, and only while the kernel sources hash to the
    recorded value."""
    paths = [p for p in os.listdir(os.path.join(ROOT, "profiles")) if p.endswith("_hbm_traffic.md")]
    assert paths
    for name in paths:
        kv = {}
        with open(os.path.join(ROOT, "profiles", name)) as f:
            for line in f:
                if line.startswith("- ") and ": " in line:
                    k, v = line[2:].split(": ", 1)
                    kv[k.strip()] = v.strip().strip("`")
        assert name == f"k_step_{kv['workload']}_{bench.config_tag(kv['config'])}_hbm_traffic.md"
        got = bench.measured_traffic(kv["workload"], kv["config"])
        if kv["kernel_source_sha256"] == bench.kernel_source_hash():
            assert got == int(kv["traffic_bytes_per_launch"])
            # traffic is at least the algorithmic bytes of one step
            assert got >= int(kv["algorithmic_bytes_per_launch"])
        else:
            assert got is None
        assert bench.measured_traffic(kv["workload"], "tile 32x32/1024") is None
        assert bench.measured_traffic("no_such_workload", kv["config"]) is None


def test_config_tags():
    assert bench.config_tag("tile 64x8/512") == "tile64x8-512"


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr
