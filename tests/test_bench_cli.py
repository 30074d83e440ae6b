"""The benchmark's command-line contract that holds without a GPU."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_a_message():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr
    assert p.stdout.strip() == ""


def test_help_lists_the_contract_flags():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--help"], capture_output=True, text=True,
                       timeout=120)
    assert p.returncode == 0
    for flag in ("--gpus", "--steps", "--warmup", "--workload"):
        assert flag in p.stdout


def test_algorithmic_op_counts():
    """The VALU roof's numerator: 56 ops per pixel for the RGB chain at the
    least work per stage, 63 in the summation order the kernels keep (shared
    pair sums in the window sums, the u8 conversion in the Gaussian),
    and the generic workload's per-stage counts (taps, window elements, one per
    point op)."""
    sys.path.insert(0, ROOT)
    import bench
    from paper_1509_04394_amd import fz
    assert bench.ops_per_px(fz.RGB_HARRIS_CHAIN) == 63
    assert bench.ops_per_px(fz.HARRIS_CHAIN) == 54
    assert bench.ops_per_px(fz.GRAD_CHAIN) == 20
    # the least work per stage (running window sums, no separate conversion)
    assert bench.ops_per_px(fz.RGB_HARRIS_CHAIN, bench.MIN_OPS) == 56
    assert bench.ops_per_px(fz.HARRIS_CHAIN, bench.MIN_OPS) == 47
    spec = bench.chain_ops("generic3")
    assert bench.ops_per_px(spec) == 9 + 1 + 9
    plan = fz.Plan(spec, 800, 600, 64)  # the three stages fuse into one group
    assert plan.segments == [2]
