"""The benchmark's command line on a host without a GPU: a request for more
than one GPU is refused with a message, before any device work."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr
    assert p.stdout == ""


def test_help_lists_the_sections():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--help"], capture_output=True, text=True,
                       timeout=120)
    assert p.returncode == 0
    for flag in ("--steps", "--warmup", "--gpus", "--no-learned", "--no-serving", "--no-multi", "--no-select"):
        assert flag in p.stdout


def test_crossover_reading():
    sys.path.insert(0, ROOT)
    import bench
    sizes = [1 << lg for lg in (8, 10, 12, 14)]
    gpu = [{"rows_per_side": n, "join_ms": 0.2} for n in sizes]
    # the oracle takes 0.05, 0.1, 0.3, 1.0 ms: the tensor path wins from between 2^10 and 2^12
    cpu = [{"rows_per_side": n, "join_ms": t} for n, t in zip(sizes, (0.05, 0.1, 0.3, 1.0))]
    x = bench.crossover(gpu, cpu, "join_ms")
    assert not x["below_sweep"] and (1 << 10) < x["rows_per_side"] < (1 << 12)
    # a dip below and back above does not count: the last crossing is taken
    cpu[0]["join_ms"] = 0.5
    assert (1 << 10) < bench.crossover(gpu, cpu, "join_ms")["rows_per_side"] < (1 << 12)
    assert bench.crossover(gpu, [dict(c, join_ms=0.01) for c in cpu], "join_ms") is None
    assert bench.crossover(gpu, [dict(c, join_ms=9.0) for c in cpu], "join_ms")["below_sweep"]
