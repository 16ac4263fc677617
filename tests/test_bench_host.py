"""Host-side checks of bench.py (no GPU): the multi-GPU refusal, the argument
surface, and that the stored HBM traffic figure belongs to the kernel sources
it was measured on (otherwise the bench reports traffic as null)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args],
                          capture_output=True, text=True, timeout=120)


def test_more_than_one_gpu_is_refused_with_a_message():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_lane_trace_refuses_other_workloads_before_any_device_work():
    r = _run("--workload", "plt_fp64_256", "--lane-trace")
    assert r.returncode == 2
    assert "--lane-trace" in r.stderr


def test_help_lists_the_workloads():
    r = _run("--help")
    assert r.returncode == 0
    for w in ("plain_fp64_256", "batch_fp32_64", "large_2048", "paper_100", "one_shot_chain",
              "plt_fp64_256", "cmesh_fp64_256", "diff_fp64_512"):
        assert w in r.stdout


def test_traffic_figure_only_for_the_sources_it_was_measured_on(monkeypatch):
    import bench
    assert bench.TRAFFIC["bytes_per_launch"] > 0
    monkeypatch.setitem(bench.TRAFFIC, "sources_sha1", bench.sources_sha1())
    assert bench.traffic_per_launch() == bench.TRAFFIC["bytes_per_launch"]
    monkeypatch.setitem(bench.TRAFFIC, "sources_sha1", "0" * 40)
    assert bench.traffic_per_launch() is None


def test_traffic_hash_covers_the_engine_sources():
    # every file the engine kernel is compiled from (its includes) is hashed
    import re

    import bench
    csrc = os.path.join(ROOT, "paper_2411_19030_amd", "csrc")
    seen, todo = set(), ["pt_host.hip"]
    while todo:
        f = todo.pop()
        if f in seen or not os.path.exists(os.path.join(csrc, f)):
            continue
        seen.add(f)
        todo += re.findall(r'#include "([^"/]+)"', open(os.path.join(csrc, f)).read())
    assert seen == set(bench.ENGINE_SOURCES)
