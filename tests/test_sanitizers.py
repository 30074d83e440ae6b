"""The host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU
only): the planner and cost-model host code (`planner.cpp`, `cost.cpp`,
`jit_layout.cpp`, with
host stand-ins for the device-side functions) driven over every fixed
sub-chain, random generic chains (temporal stages included), configuration
overrides, the partition model and learned planning; and the oracle's C code
driven over small and degenerate volumes and the tracker.  Built with g++/gcc
(host code only; no device code is instrumented)."""
import json
import os
import shutil
import struct
import subprocess

import numpy as np
import pytest

from paper_1509_04394_amd import costmodel, fz, synth

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_1509_04394_amd", "csrc")
SAN = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")


def have(tool):
    return shutil.which(tool) is not None


def write_chains(path, seeds):
    """Random generic chains (the learned-cost recipe) plus temporal stages, as
    text: n, then per stage op rx ry rt a b c n_weights weights..."""
    ops = {"stencil": fz.OPS["stencil"], "box": fz.OPS["box"], "point": fz.OPS["point"], "iir": fz.OPS["iir"]}
    with open(path, "w") as f:
        for sd in seeds:
            spec = synth.random_chain(sd)
            if sd % 3 == 0:  # temporal stages too
                spec = [("iir", 0.25)] + spec[:5] + [("stencil", 1, 0, np.full((3, 1, 3), 1 / 9.0, np.float32))]
            f.write(f"{len(spec)}\n")
            for st in spec:
                if st[0] == "point":
                    f.write(f"{ops['point']} 0 0 0 {fz.POINT_KINDS[st[1]]} {st[2]} {st[3]} 0\n")
                elif st[0] == "iir":
                    f.write(f"{ops['iir']} 0 0 -1 {st[1]} 0 0 0\n")
                elif st[0] == "box":
                    f.write(f"{ops['box']} {st[1]} {st[2]} 0 0 0 0 0\n")
                else:
                    w = np.asarray(st[3], np.float32)
                    rt = w.shape[0] - 1 if w.ndim == 3 else 0
                    f.write(f"{ops['stencil']} {st[1]} {st[2]} {rt} 0 0 0 {w.size} " +
                            " ".join(repr(float(v)) for v in w.ravel()) + "\n")


@pytest.mark.skipif(not have("g++"), reason="no host compiler")
def test_planner_under_sanitizers(tmp_path):
    exe = str(tmp_path / "planner_driver")
    srcs = [os.path.join(HERE, "sanitize", "planner_driver.cpp"), os.path.join(HERE, "sanitize", "device_stubs.cpp"),
            os.path.join(CSRC, "planner.cpp"), os.path.join(CSRC, "cost.cpp"),
            os.path.join(CSRC, "jit_layout.cpp")]
    subprocess.check_call(["g++", "-std=c++17", *SAN, f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}", *srcs,
                           "-o", exe])
    chains = str(tmp_path / "chains.txt")
    write_chains(chains, range(5000, 5030))
    weights = str(tmp_path / "weights.bin")
    params, _ = costmodel.load_weights()
    with open(weights, "wb") as f:
        f.write(struct.pack(f"{len(params)}f", *params))
    r = subprocess.run([exe, chains, weights], capture_output=True, text=True, env=ENV, timeout=600)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), (r.stdout[-2000:], r.stderr[-4000:])


@pytest.mark.skipif(not have("gcc"), reason="no host compiler")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    subprocess.check_call(["gcc", "-std=c99", *SAN, os.path.join(HERE, "sanitize", "oracle_driver.c"),
                           os.path.join(ROOT, "oracle", "oracle.c"), os.path.join(ROOT, "oracle", "track.c"),
                           "-lm", "-lpthread", "-o", exe])
    r = subprocess.run([exe], capture_output=True, text=True, env=ENV, timeout=600)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), (r.stdout[-2000:], r.stderr[-4000:])
