"""Build the gfx950 HIP library libfoamlbm.so in-tree with hipcc.

Each translation unit is compiled to an object in parallel, then linked.  A
stamp file beside the library records a hash of the sources it was built from
(csrc/ and include/); the binding refuses a library whose stamp differs from
the sources in the tree.
"""
import glob
import hashlib
import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRCS = [os.path.join(HERE, "csrc", f) for f in ("foamlbm.hip", "batch.hip", "server.hip")]
LIB = os.path.join(HERE, "libfoamlbm.so")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # packed FP32 instructions stay off: the compiler may not form them
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def source_files():
    """Every file the library is built from, in a fixed order."""
    files = glob.glob(os.path.join(HERE, "csrc", "*.hip")) + glob.glob(os.path.join(HERE, "csrc", "*.hpp"))
    files += glob.glob(os.path.join(ROOT, "include", "*.h"))
    return sorted(files)


def source_hash(defines=()):
    h = hashlib.sha256()
    for p in source_files():
        h.update(os.path.relpath(p, ROOT).encode())
        with open(p, "rb") as fh:
            h.update(fh.read())
    for d in defines:
        h.update(b"-D" + d.encode())
    return h.hexdigest()[:32]


def stamp_of(lib):
    try:
        with open(lib + ".srchash") as fh:
            return fh.read().strip()
    except OSError:
        return None


def build(verbose: bool = False, out: str = LIB, defines=()) -> str:
    """Compile the library to `out`; `defines` are extra -D options (the
    compile-time switches of the kernels, e.g. FLB_ST_CPOL=2)."""
    dflags = [f"-D{d}" for d in defines]
    with tempfile.TemporaryDirectory(prefix="flb_build_") as tmp:
        objs = [os.path.join(tmp, os.path.basename(s) + ".o") for s in SRCS]
        cmds = [["hipcc", *FLAGS, *dflags, "-c", s, "-o", o] for s, o in zip(SRCS, objs)]

        def run(cmd):
            if verbose:
                print(" ".join(cmd), flush=True)
            subprocess.run(cmd, check=True)

        with ThreadPoolExecutor(max_workers=len(cmds)) as ex:
            for f in [ex.submit(run, c) for c in cmds]:
                f.result()
        run(["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", out + ".tmp"])
    os.replace(out + ".tmp", out)
    with open(out + ".srchash", "w") as fh:
        fh.write(source_hash(defines) + "\n")
    return out


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
