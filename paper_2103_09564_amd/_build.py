"""Build librwseg.so (all HIP sources of the package) for gfx950 with hipcc.

Each source compiles to its own object in a private temporary directory
(the sources share no device code, so no relocatable device code is needed),
in parallel, and the objects are linked into the shared library.
"""

import os
import shutil
import subprocess
import tempfile
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "librwseg.so")

SOURCES = ["capi.hip", "pcg.hip", "domain.hip", "resident.hip", "hier.hip", "probe.hip"]

HIPCC_FLAGS = [
    "-O3", "--offload-arch=gfx950", "-std=c++17", "-fPIC",
    # packed FP32 instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def hipcc():
    exe = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(exe):
        raise RuntimeError("hipcc not found (ROCm is required to build librwseg)")
    return exe


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + " ".join(cmd) + "\n" + res.stdout + res.stderr)


def build_library(verbose=False, jobs=None):
    """Compile librwseg.so in-tree; always rebuilds.  Returns the path."""
    srcs = list(SOURCES)
    jobs = jobs or min(len(srcs), max(1, min(os.cpu_count() or 1, 16)))
    with tempfile.TemporaryDirectory(prefix="rwseg_build_") as tmpd:
        objs = [os.path.join(tmpd, os.path.splitext(s)[0] + ".o") for s in srcs]
        cmds = [[hipcc()] + HIPCC_FLAGS + ["-I" + INCLUDE, "-I" + CSRC, "-c",
                                           os.path.join(CSRC, s), "-o", o]
                for s, o in zip(srcs, objs)]
        with ThreadPoolExecutor(max_workers=jobs) as ex:
            for f in [ex.submit(_run, c, verbose) for c in cmds]:
                f.result()
        tmp = LIB + ".tmp"
        _run([hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC"] + objs + ["-o", tmp], verbose)
        os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build_library(verbose=True))
