"""Build libmra.so in-tree with hipcc for gfx950.

Usage: python -m paper_1507_01888_amd.build   (or build() from Python)
"""
import concurrent.futures
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libmra.so")
BUILD_DIR = os.path.join(HERE, "_build")

SOURCES = ["host_numerics.cpp", "tree_project.cpp", "apply_ns.cpp", "capi.cpp", "wavelet.cpp", "kernels.hip"]

COMMON = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
          # packed FP32 instructions are kept out of all device code
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wno-unused-result"]


def _hipcc():
    exe = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(exe):
        raise RuntimeError("hipcc not found")
    return exe


# Device code: matrix-core results and accumulators in VGPRs rather than AGPRs.  The BF16
# tier kernel converts every matrix-core result with vector instructions, which read only
# VGPRs; with the compiler's default choice it spent ~1,300 AGPR-to-VGPR moves per loop
# iteration (measured: 7% faster BF16 kernel, 1.5% faster FP64 k=14 kernel with this form).
DEVICE_EXTRA = {"kernels.hip": ["-mllvm", "--amdgpu-mfma-vgpr-form"]}


def _compile(src):
    obj = os.path.join(BUILD_DIR, os.path.splitext(src)[0] + ".o")
    cmd = [_hipcc()] + COMMON + DEVICE_EXTRA.get(src, []) + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("compiling %s failed:\n%s\n%s" % (src, " ".join(cmd), r.stderr))
    return obj


def build(verbose=False):
    """Compile every source and link libmra.so (always rebuilds)."""
    os.makedirs(BUILD_DIR, exist_ok=True)
    with concurrent.futures.ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = OUT + ".tmp"
    # --no-undefined: a kernel whose host stub was not emitted fails here, not at load time
    cmd = [_hipcc(), "-shared", "-fPIC", "--offload-arch=gfx950", "-Wl,--no-undefined", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("linking libmra.so failed:\n%s\n%s" % (" ".join(cmd), r.stderr))
    os.replace(tmp, OUT)
    if verbose:
        print("built", OUT)
    return OUT


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
