"""Host-side pieces of bench.py: the one-GPU guard, the kernel table and the
traffic figure read from the committed counter summary."""
import hashlib
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_kernel_table_means():
    t = {"a": {"ms": 12.0, "launches": 6}, "b": {"ms": 0.0, "launches": 0}}
    kt = bench.kernel_table(t, 3)
    assert kt == {"a": {"ms_per_step": 4.0, "launches_per_step": 2.0, "ms_per_launch": 2.0}}


def test_traffic_follows_the_kernel_source_hash():
    sha = hashlib.sha256(open(bench.MATCH_SRC, "rb").read()).hexdigest()
    recorded = None
    for line in open(bench.TRAFFIC_FILE):
        if line.strip().startswith("- match.hip sha256:"):
            recorded = line.split(":", 1)[1].strip()
    t = bench.measured_traffic()
    if recorded == sha:
        assert t is not None and t > 48777104          # above the algorithmic bytes
    else:
        assert t is None


def test_describe_valu_count_follows_the_kernel_source_hash():
    sha = hashlib.sha256(open(bench.DESC_SRC, "rb").read()).hexdigest()
    recorded = None
    for line in open(bench.DESC_COUNTERS_FILE):
        if line.strip().startswith("- describe.hip sha256:"):
            recorded = line.split(":", 1)[1].strip()
    n = bench.describe_valu_instructions()
    if recorded == sha:
        assert n is not None and n > 1e6
    else:
        assert n is None


def test_committed_figure_reads_key_lines(tmp_path):
    src = tmp_path / "k.hip"
    src.write_text("kernel")
    sha = hashlib.sha256(b"kernel").hexdigest()
    f = tmp_path / "s.md"
    f.write_text(f"# t\n\n- k.hip sha256: {sha}\n- figure: 12.5\n")
    assert bench.committed_figure(str(f), str(src), "k.hip sha256", "figure") == 12.5
    assert bench.committed_figure(str(f), str(src), "k.hip sha256", "other") is None
    src.write_text("changed")
    assert bench.committed_figure(str(f), str(src), "k.hip sha256", "figure") is None
