"""Build libtnrg.so for gfx950 with hipcc (in-tree, no JIT cache)."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB_DIR = os.path.join(HERE, "_lib")
LIB_PATH = os.path.join(LIB_DIR, "libtnrg.so")
SOURCES = [os.path.join(HERE, "csrc", "tnrg_lib.hip"), os.path.join(HERE, "csrc", "tnrg_server.cpp")]
HEADERS = [os.path.join(HERE, "csrc", "tnrg_device.hpp"),
           os.path.join(HERE, "csrc", "tnrg_common.hpp"),
           os.path.join(HERE, "csrc", "tnrg_kernels.inc"),
           os.path.join(ROOT, "include", "tnrg.h")]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("TNRG_ARCH", "gfx950")

FLAGS = [
    "-O3", "-std=c++17", "-shared", "-fPIC",
    f"--offload-arch={ARCH}",
    # packed fp32 instructions are disabled for all device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-fno-gpu-rdc",
    "-I", os.path.join(ROOT, "include"),
    "-I", os.path.join(HERE, "csrc"),
]


def build(verbose: bool = False) -> str:
    """Compile the HIP library; returns the path of the shared object."""
    os.makedirs(LIB_DIR, exist_ok=True)
    tmp = LIB_PATH + ".tmp"
    cmd = [HIPCC] + FLAGS + SOURCES + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed to build libtnrg.so")
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


if __name__ == "__main__":
    print(build(verbose=True))
