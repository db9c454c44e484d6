"""The library's host code under AddressSanitizer and
UndefinedBehaviorSanitizer: every HIP source is compiled with the host pass
instrumented (-Xarch_host before each -fsanitize=, so the device code is
built as usual), and the driver tests/native/abi_sanitize_main.c, built with
the same sanitizers, calls every entry point with invalid arguments and
every size query with sizes up to INT32_MAX. No recovery: any invalid
access, leak or undefined operation in the argument checks, the workspace
arithmetic or the batch planner's rejection paths fails the run. (With a
GPU, `abi_sanitize gpu` runs every entry point on small systems as well.)"""
import glob
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANG = "/opt/rocm/llvm/bin/clang"

SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]


def build_sanitized(out):
    """The library with its host pass instrumented, and the driver; returns
    the driver's path."""
    csrc = os.path.join(ROOT, "paper_1909_06623_amd", "csrc")
    inc = ["-I", os.path.join(ROOT, "include"), "-I", csrc]
    flags = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-ffp-contract=off",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", *SAN]
    srcs = sorted(glob.glob(os.path.join(csrc, "*.hip")))
    objs = [os.path.join(out, os.path.basename(s)[:-4] + ".o") for s in srcs]

    def cc(so):
        subprocess.run([HIPCC, *flags, *inc, "-c", "-o", so[1], so[0]], check=True,
                       capture_output=True, text=True, timeout=600)

    with ThreadPoolExecutor(max(1, min(len(srcs), os.cpu_count() or 1))) as ex:
        list(ex.map(cc, zip(srcs, objs)))
    lib = os.path.join(out, "libscgpu.so")
    subprocess.run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *SAN, "-o", lib, *objs],
                   check=True, capture_output=True, text=True, timeout=600)
    exe = os.path.join(out, "abi_sanitize")
    subprocess.run([CLANG, "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"),
                    "-I", "/opt/rocm/include", os.path.join(HERE, "native", "abi_sanitize_main.c"),
                    lib, "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,$ORIGIN",
                    "-Wl,-rpath,/opt/rocm/lib", "-o", exe],
                   check=True, capture_output=True, text=True, timeout=300)
    return exe


@pytest.mark.timeout(900)
@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANG)),
                    reason="needs hipcc and ROCm's clang")
def test_library_host_code_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    exe = build_sanitized(str(tmp_path))
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "host checks: ok" in r.stdout and "all ok" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
