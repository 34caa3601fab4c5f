"""Build libunihenn.so for gfx950 with hipcc (in-tree, no JIT cache).

Every HIP source under csrc/ is compiled to an object in _build/ (in
parallel) and linked into paper_2402_03060_amd/libunihenn.so.
`python -m paper_2402_03060_amd.build int_rates` builds the integer
issue-rate microbenchmark instead.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libunihenn.so")
ARCH = os.environ.get("UNIHENN_ARCH", "gfx950")

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-Wall", "-Wno-unused-function",
]


def sources() -> list[str]:
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = ["hipcc", *FLAGS, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stderr}")
    errs = [l for l in r.stderr.splitlines() if "warning" in l and "packed-fp32-ops" not in l]
    if errs:
        sys.stderr.write("\n".join(errs[:20]) + "\n")
    return obj


def build(jobs: int = 8) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()
    with cf.ThreadPoolExecutor(max_workers=min(jobs, len(srcs))) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp"
    subprocess.check_call(["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp])
    os.replace(tmp, LIB)
    return LIB


def build_int_rates() -> str:
    """The integer issue-rate microbenchmark (microbench/int_rates.cpp), built
    on demand next to its source."""
    src = os.path.join(PKG, "microbench", "int_rates.cpp")
    exe = os.path.join(PKG, "microbench", "int_rates")
    subprocess.check_call(["hipcc", f"--offload-arch={ARCH}", "-O3", "-Xclang", "-target-feature", "-Xclang",
                           "-packed-fp32-ops", src, "-o", exe])
    return exe


if __name__ == "__main__":
    print(build_int_rates() if sys.argv[1:] == ["int_rates"] else build())
