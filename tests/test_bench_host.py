"""Host checks of bench.py (no GPU): the script parses and imports, its
traffic files name the kernel sources they were taken from, and it refuses a
multi-GPU run with a message."""
import ast
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_parses_and_imports():
    src = open(os.path.join(ROOT, "bench.py")).read()
    ast.parse(src)
    sys.path.insert(0, ROOT)
    import bench  # noqa: F401  (module level only: no GPU work at import)
    assert callable(bench.main)


def test_traffic_files_carry_a_source_digest():
    sys.path.insert(0, ROOT)
    import bench
    for path in (bench.TRAFFIC_FILE, bench.FIXED_TRAFFIC_FILE):
        kv = dict(line.split(": ", 1) for line in open(path).read().splitlines()
                  if line and not line.startswith("#"))
        assert len(kv["kernel_source_sha256"]) == 64
        assert float(kv["traffic_bytes_per_launch"]) > 0


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)
