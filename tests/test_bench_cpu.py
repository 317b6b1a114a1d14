"""CPU checks of the benchmark's host logic (no GPU needed)."""

import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]


def test_source_hash_ignores_comments_only():
    a = "double f(double x) { return x * 2.0; } // twice\n/* block\n comment */"
    b = "double f(double x)\n{\n    return x * 2.0;\n}\n"
    c = "double f(double x) { return x * 3.0; }"
    assert bench._code_only(a) == bench._code_only(b)
    assert bench._code_only(a) != bench._code_only(c)


def test_source_hash_covers_the_plane_padding():
    """The padding the host gives every plane is part of the hash (it moves
    the kernels' addresses and so their traffic)."""
    import re

    src = open(os.path.join(ROOT, "paper_1505_02037_amd", "csrc", "lb_api.hip")).read()
    assert re.search(r"constexpr size_t kPlanePad = \d+;", src)


def test_traffic_summary_is_used_only_for_matching_sources():
    path = os.path.join(ROOT, "profiles", "traffic_fp64_step.json")
    d = json.load(open(path))
    t = bench.measured_traffic(256 ** 3, "fp64")
    if d["kernel_source_sha"] == bench.kernel_source_hash():
        assert abs(t / 256 ** 3 - d["bytes_per_site_per_step"]) < 1e-6
    else:
        assert t is None


def test_cpu_case_runs_the_oracle_alone():
    env = dict(os.environ, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--cpu-case", "c1", "--single"],
                       capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stderr
    d = json.loads(r.stdout.strip().splitlines()[-1])
    assert d["threads"] == 1 and d["steps"] == 1000 and d["site_updates_per_s"] > 0
