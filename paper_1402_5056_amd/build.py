"""Compile the h2lr HIP library for gfx950 (in-tree shared object)."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libh2lr.so")
SOURCES = [os.path.join(HERE, "csrc", "api.hip")]
DEPS = [os.path.join(HERE, "csrc", f) for f in ("api.hip", "tasks.hip", "dense.h", "common.h")] + \
    [os.path.join(ROOT, "include", "h2lr.h")]


def hipcc_command(out=LIB, arch="gfx950"):
    return ["/opt/rocm/bin/hipcc", f"--offload-arch={arch}", "-O3", "-std=c++17", "-fPIC", "-shared",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc"),
            *SOURCES, "-o", out]


def build(verbose=True, out=LIB):
    """Always recompiles, also when a built library is present."""
    cmd = hipcc_command(out + ".tmp")
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed")
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    build(out=os.path.abspath(sys.argv[1]) if len(sys.argv) > 1 else LIB)
