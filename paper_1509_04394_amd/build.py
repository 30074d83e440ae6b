"""Build the fz C-ABI library (libfz.so) for gfx950 in-tree.

Every HIP translation unit is compiled with hipcc for gfx950 only, with
floating-point contraction off (so each kernel variant evaluates the same
expressions with the same roundings) and packed FP32 instructions disabled.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libfz.so")
BUILD_DIR = os.path.join(ROOT, "_build")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
COMMON = ["-O3", "-std=c++17", "-fPIC", "-ffp-contract=off", "-Wall", "-Wno-unused-function",
          f"-I{os.path.join(ROOT, 'include')}"]
HIP_FLAGS = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-munsafe-fp-atomics"]


def sources():
    hip = sorted(f for f in os.listdir(CSRC) if f.endswith(".hip"))
    cpp = sorted(f for f in os.listdir(CSRC) if f.endswith(".cpp"))
    return hip, cpp


def _compile(src: str, obj: str, hip: bool) -> tuple[str, int, str]:
    cmd = [HIPCC] + COMMON + (HIP_FLAGS + ["-x", "hip"] if hip else []) + ["-c", src, "-o", obj]
    p = subprocess.run(cmd, capture_output=True, text=True)
    out = p.stdout + p.stderr
    # hipcc's host pass does not know the packed-fp32 feature name; that note is harmless
    out = "\n".join(l for l in out.splitlines() if "packed-fp32-ops" not in l)
    return src, p.returncode, out


def _stale(obj: str, newest_source: float) -> bool:
    return not os.path.exists(obj) or os.path.getmtime(obj) < newest_source


def build(jobs: int | None = None, verbose: bool = False, incremental: bool = False) -> str:
    """Compile every translation unit and link libfz.so.  With `incremental`,
    objects newer than every source and header are reused (development aid)."""
    os.makedirs(BUILD_DIR, exist_ok=True)
    hip, cpp = sources()
    tasks = [(os.path.join(CSRC, f), os.path.join(BUILD_DIR, f + ".o"), True) for f in hip]
    tasks += [(os.path.join(CSRC, f), os.path.join(BUILD_DIR, f + ".o"), False) for f in cpp]
    all_tasks = tasks
    if incremental:
        deps = [os.path.join(CSRC, f) for f in os.listdir(CSRC)] + [os.path.join(ROOT, "include", "fz.h")]
        newest = max(os.path.getmtime(d) for d in deps)
        tasks = [t for t in tasks if _stale(t[1], newest)]
    jobs = jobs or min(max(len(tasks), 1), max(1, (os.cpu_count() or 4)))
    with cf.ThreadPoolExecutor(jobs) as ex:
        results = list(ex.map(lambda t: _compile(*t), tasks))
    failed = [r for r in results if r[1] != 0]
    tasks = all_tasks
    for src, rc, out in results:
        if out.strip() and (verbose or rc != 0):
            print(f"--- {os.path.basename(src)} (rc={rc})\n{out}", file=sys.stderr)
    if failed:
        raise RuntimeError("compilation failed: " + ", ".join(os.path.basename(f[0]) for f in failed))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + [t[1] for t in tasks] + ["-lhiprtc"]
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


def clean():
    shutil.rmtree(BUILD_DIR, ignore_errors=True)


if __name__ == "__main__":
    build(verbose="-v" in sys.argv, incremental="--incremental" in sys.argv)
    print(LIB)
