"""Host logic of bench.py (no GPU): the algorithmic flop count behind every
TFLOP/s figure, the gate that reports profiled HBM traffic only for the
kernel source the counters were taken on, and the refusal of a multi-GPU run."""
import importlib.util
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_block_flops_whole_solve(bench):
    # C2: H = 2000 block updates of b = 8 at s = 64 -> 31 outer iterations of
    # 64 blocks and a last one of 16; every block update costs 2 m n b
    m, n, b = 20000, 512, 8
    assert bench.block_flops(2000, 64, b, m, n) == 2 * m * n * b * 2000


def test_block_flops_every_eighth(bench):
    # outer iterations k = 0, 8, 16, 24 (all of 64 blocks); k = 31 is not counted
    m, n, b = 20000, 512, 8
    assert bench.block_flops(2000, 64, b, m, n, every=8) == 4 * 2 * m * n * 64 * b
    # a ragged last iteration that falls on k % 8 == 0 counts its own width
    assert bench.block_flops(8 * 10 + 3, 10, 1, 7, 5, every=8) == 2 * 7 * 5 * (10 + 3)


def test_profiled_traffic_follows_the_source(bench, tmp_path):
    src = [tmp_path / "k.hip", tmp_path / "h.hpp"]
    src[0].write_text("kernel body\n")
    src[1].write_text("header\n")
    digest = bench.source_digest([str(p) for p in src])
    prof = tmp_path / "prof.txt"
    prof.write_text("# summary\ntraffic_bytes_per_launch: 123000\n"
                    f"source_sha256: {digest}\n")
    assert bench.profiled_traffic(str(prof), [str(p) for p in src]) == 123000.0
    # any change to either file voids the figure
    src[1].write_text("header, edited\n")
    assert bench.profiled_traffic(str(prof), [str(p) for p in src]) is None
    # so does a missing profile
    assert bench.profiled_traffic(str(tmp_path / "none.txt"), [str(p) for p in src]) is None


def test_multi_gpu_run_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""
