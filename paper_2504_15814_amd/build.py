"""Build libfacetransfer.so (HIP, gfx950) in-tree with hipcc.

Usage: python -m paper_2504_15814_amd.build [-v]
"""

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIBDIR = os.path.join(HERE, "lib")
LIBNAME = "libfacetransfer.so"
INCLUDE = os.path.join(ROOT, "include")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
# Packed FP32 instructions are disabled for all device code.
NO_PACKED_FP32 = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
COMMON = ["-std=c++17", "-fPIC", "-O3", "-I", INCLUDE, "-I", CSRC, "-Wall", "-Wno-unused-function"]

DEVICE_SOURCES = ["ft_kernels.hip", "ft_mfma.hip", "ft_plan.hip", "ft_patch.hip"]
HOST_SOURCES = ["ft_builder.cpp", "ft_api.cpp"]


def lib_path():
    return os.path.join(LIBDIR, LIBNAME)


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError(f"command failed ({res.returncode}): {' '.join(cmd)}")
    return res


def build(verbose=False, jobs=None):
    """Compile every source (in parallel, `jobs` at a time) and link the
    shared library; returns its path."""
    from concurrent.futures import ThreadPoolExecutor

    obj_dir = os.path.join(HERE, "_build")
    os.makedirs(obj_dir, exist_ok=True)
    os.makedirs(LIBDIR, exist_ok=True)
    cmds, objs = [], []
    for src in DEVICE_SOURCES:
        obj = os.path.join(obj_dir, src + ".o")
        cmds.append([HIPCC, "-x", "hip", f"--offload-arch={ARCH}", *COMMON, *NO_PACKED_FP32, "-c",
                     os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    for src in HOST_SOURCES:
        obj = os.path.join(obj_dir, src + ".o")
        cmds.append([HIPCC, *COMMON, *NO_PACKED_FP32, "-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    jobs = jobs or min(len(cmds), os.cpu_count() or 1, 8)
    with ThreadPoolExecutor(max_workers=jobs) as pool:
        for fut in [pool.submit(_run, c, verbose) for c in cmds]:
            fut.result()
    tmp = lib_path() + ".tmp"
    _run([HIPCC, "-shared", f"--offload-arch={ARCH}", "-fPIC", *objs, "-o", tmp], verbose)
    os.replace(tmp, lib_path())
    return lib_path()


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
