"""Build libfskmc.so for gfx950 with hipcc (in-tree, next to this file)."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libfskmc.so")
SOURCES = [os.path.join(HERE, "csrc", "fskmc_kernels.hip"), os.path.join(HERE, "csrc", "fskmc_noalloc.hip"),
           os.path.join(HERE, "csrc", "fskmc_host.cpp")]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# -ffp-contract=off: the decision path must round like the CPU statement of the
# scheme (no fused multiply-add).  Packed FP32 instructions are disabled.  The
# iterative ILP scheduler orders the kernels' dependent chains for latency
# (the resident sweep's window: 1.7% shorter than the default scheduler's, the
# same bits); it changes instruction order only.
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=off",
         "-fno-fast-math", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-mllvm", "-amdgpu-sched-strategy=iterative-ilp",
         "-I", os.path.join(ROOT, "include"), "-Wall", "-Wno-unused-function"]


def build(verbose=False, out=None, extra_flags=()):
    """Build libfskmc.so in-tree, or a variant at `out` with `extra_flags`
    (e.g. host-side sanitizers, each after -Xarch_host)."""
    target = out or LIB
    tmp = target + ".tmp%d" % os.getpid()
    cmd = [HIPCC] + FLAGS + list(extra_flags) + ["-o", tmp] + SOURCES
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building libfskmc")
    os.replace(tmp, target)
    return target


if __name__ == "__main__":
    print(build(verbose=True))
