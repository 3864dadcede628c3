"""Host-side pieces of bench.py: the one-GPU guard, the kernel table, the
traffic figure read from the committed counter summary, the support-visit
count and the tile-pair geometry."""
import hashlib
import math
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

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
    if os.path.exists(bench.TRAFFIC_FILE):
        for line in open(bench.TRAFFIC_FILE):
            if line.strip().startswith("- match.hip sha256:"):
                recorded = line.split(":", 1)[1].strip()
    t = bench.measured_traffic()
    if recorded == sha:
        assert t is not None and t > 1e8          # above any launch's algorithmic bytes
    else:
        assert t is None


def test_support_visits_and_sides():
    ws = bench.subregion_sides([16, 32, 64, 128])
    assert np.allclose(ws, [4.0, math.sqrt(32), 8.0, math.sqrt(128)], rtol=1e-14)
    v = bench.support_visits([16], [4.0])
    # square of side 20 (400) + the 113 integer points of the radius-6 disc
    assert v == [400.0 + 113]


def test_pair_geometry_of_the_grid():
    class T:
        order = np.arange(9)
    nb, far = bench.pair_geometry(T)
    assert len(nb) == 12 and len(far) == 16       # 8 diagonal pairs are neither
    assert (0, 1) in nb and (0, 3) in nb and (0, 2) in far and (0, 4) not in far + nb


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
