"""Host-side logic of bench.py (no GPU): the one-GPU guard, the rule that
HBM traffic is reported only while the kernel sources match the profiled
ones, and the percentile helper."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_traffic_follows_the_source_hash(tmp_path):
    h = bench.kernel_source_hash(bench.HYPERBOLIC_SOURCES)
    body = "Kernel source hash: `%s`\n\ntraffic_bytes_per_launch k_hyperbolic<double>: 1073926819   (ratio)\n"
    good = tmp_path / "good.md"
    good.write_text(body % h)
    stale = tmp_path / "stale.md"
    stale.write_text(body % ("0" * 16))
    assert bench.counted_traffic(str(good), "k_hyperbolic<double>", bench.HYPERBOLIC_SOURCES) == 1073926819
    assert bench.counted_traffic(str(stale), "k_hyperbolic<double>", bench.HYPERBOLIC_SOURCES) is None
    assert bench.counted_traffic(str(tmp_path / "missing.md"), "k_hyperbolic<double>",
                                 bench.HYPERBOLIC_SOURCES) is None
    # the hash covers every listed source: a different set hashes differently
    assert bench.kernel_source_hash(bench.QUANTILE_SOURCES) != h


def test_committed_profiles_parse():
    """Both committed counter summaries carry a hash and a traffic line that
    the bench reads (the figure itself is null once a source changes)."""
    for prof, kern, files, algo in (
            ("quantile_mixture_2e28_hbm_counters.md", "k_hybrid<double>", bench.QUANTILE_SOURCES, 16 << 28),
            ("hyperbolic_exp_2e26_hbm_counters.md", "k_hyperbolic<double>", bench.HYPERBOLIC_SOURCES, 16 << 26)):
        text = open(os.path.join(ROOT, "profiles", prof)).read()
        assert "Kernel source hash: `" in text and ("traffic_bytes_per_launch %s: " % kern) in text
        t = bench.counted_traffic(prof, kern, files)
        if t is not None:
            assert algo <= t < 1.01 * algo


def test_percentile():
    xs = [5.0, 1.0, 4.0, 2.0, 3.0]
    assert bench.percentile(xs, 50) == 3.0
    assert bench.percentile(xs, 99) == 5.0
    assert bench.percentile(xs, 0) == 1.0
    assert bench.percentile([], 50) is None
