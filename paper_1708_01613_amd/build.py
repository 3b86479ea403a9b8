"""Build the gfx950 HIP library libfoamlbm.so in-tree with hipcc."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRCS = [os.path.join(HERE, "csrc", f) for f in ("foamlbm.hip", "batch.hip", "server.hip")]
LIB = os.path.join(HERE, "libfoamlbm.so")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # packed FP32 instructions stay off: the compiler may not form them
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def build(verbose: bool = False, out: str = LIB, defines=()) -> str:
    """Compile the library to `out`; `defines` are extra -D options (the
    compile-time switches of the kernels, e.g. FLB_ST_CPOL=2)."""
    cmd = ["hipcc", *FLAGS, *[f"-D{d}" for d in defines], *SRCS, "-o", out + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


PROBE = os.path.join(HERE, "copy_probe")


def build_probe(verbose: bool = False) -> str:
    """Compile the standalone copy-bandwidth probe (csrc/copy_probe.hip) to
    `copy_probe` beside this file: the practical HBM ceilings by access width."""
    cmd = ["hipcc", "--offload-arch=gfx950", "-O3", "-std=c++17", "-Xclang", "-target-feature", "-Xclang",
           "-packed-fp32-ops", os.path.join(HERE, "csrc", "copy_probe.hip"), "-o", PROBE]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return PROBE


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
