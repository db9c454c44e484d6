"""Build the gfx950 HIP library ``paper_1909_06623_amd/libscgpu.so``.

Every HIP source under ``csrc/`` is compiled for ``--offload-arch=gfx950``
(one hipcc per source, in parallel, objects under ``_build/``) and linked
into one shared library. Floating-point contraction is disabled so that the
pair-geometry arithmetic rounds exactly as written, and packed-FP32
instruction selection is turned off.
"""
import glob
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
LIB = os.path.join(PKG, "libscgpu.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-ffp-contract=off", "-Wall", "-Wno-unused-function",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def sources():
    return sorted(glob.glob(os.path.join(PKG, "csrc", "*.hip")))


def _compile(src, obj, verbose):
    flags = [a for a in FLAGS if a != "-shared"]
    cmd = [HIPCC, *flags, "-c", "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(PKG, "csrc"), "-o", obj, src]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return obj


def build(verbose=False, jobs=None):
    """Compile every source to an object (in parallel) and link the shared
    library. Always recompiles."""
    from concurrent.futures import ThreadPoolExecutor
    out = os.path.join(PKG, "_build")
    os.makedirs(out, exist_ok=True)
    srcs = sources()
    objs = [os.path.join(out, os.path.basename(f)[:-4] + ".o") for f in srcs]
    for stale in set(glob.glob(os.path.join(out, "*.o"))) - set(objs):
        os.remove(stale)
    jobs = jobs or min(len(srcs), max(1, min(16, os.cpu_count() or 1)))
    with ThreadPoolExecutor(jobs) as ex:
        list(ex.map(lambda so: _compile(so[0], so[1], verbose), zip(srcs, objs)))
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", LIB + ".tmp", *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
