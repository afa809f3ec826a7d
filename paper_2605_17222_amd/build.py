"""Build libckks_lt.so for gfx950 with hipcc (in-tree)."""
from __future__ import annotations

import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libckks_lt.so")
ARCH = os.environ.get("CKKS_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    "--offload-arch=" + ARCH,
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    # no packed FP32 instructions anywhere
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))


def _jobs() -> int:
    try:
        n = int(os.environ.get("MAX_JOBS", "0"))
    except ValueError:
        n = 0
    return max(1, min(n or (os.cpu_count() or 1), 16))


def build(verbose: bool = False) -> str:
    """Compiles every source to an object in parallel, then links the library."""
    import tempfile
    from concurrent.futures import ThreadPoolExecutor

    tmp = LIB + ".tmp%d" % os.getpid()
    with tempfile.TemporaryDirectory(prefix="ckks_build_") as od:
        srcs = sources()
        objs = [os.path.join(od, os.path.basename(f) + ".o") for f in srcs]
        compile_flags = [f for f in FLAGS if f != "-shared"]

        def run(cmd):
            if verbose:
                print(" ".join(cmd), flush=True)
            return subprocess.run(cmd, capture_output=True, text=True)

        with ThreadPoolExecutor(_jobs()) as ex:
            rs = list(ex.map(run, [["hipcc"] + compile_flags + ["-c", f, "-o", o] for f, o in zip(srcs, objs)]))
        rs.append(run(["hipcc"] + FLAGS + objs + ["-o", tmp]) if all(r.returncode == 0 for r in rs) else rs[0])
        for r in rs:
            if r.returncode != 0:
                sys.stderr.write(r.stdout + r.stderr)
                raise RuntimeError("hipcc failed building %s" % LIB)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
