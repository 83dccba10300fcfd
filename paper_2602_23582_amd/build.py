"""Build the RBSOG HIP library (librbsog.so) for gfx950 with hipcc, in-tree."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "librbsog.so")
PROBE_LIB = os.path.join(HERE, "libvaluprobe.so")
SOURCES = ["kernels.hip", "setup.cpp", "system.cpp", "api.cpp", "batch_api.cpp", "server.cpp", "npt.cpp", "noalloc.cpp"]
ARCH = os.environ.get("RBSOG_OFFLOAD_ARCH", "gfx950")


def hipcc_flags():
    return [
        "-x", "hip", f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
        # no packed FP32 instructions: every FP32 operation is issued unpacked
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-Wall", "-Wno-unused-function",
        "-I", os.path.join(ROOT, "include"), "-I", CSRC,
    ]


def build_library(verbose: bool = False, extra=None) -> str:
    objs = []
    build_dir = os.path.join(HERE, "_build")
    os.makedirs(build_dir, exist_ok=True)
    for src in SOURCES:
        obj = os.path.join(build_dir, src + ".o")
        cmd = ["hipcc", "-c", *hipcc_flags(), *(extra or []), os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        objs.append(obj)
    cmd = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", LIB + ".tmp", *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    # the issue-rate probe behind the ALU roofline (separate library)
    cmd = ["hipcc", *hipcc_flags(), "-shared", os.path.join(CSRC, "valu_probe.hip"), "-o", PROBE_LIB + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(PROBE_LIB + ".tmp", PROBE_LIB)
    return LIB


if __name__ == "__main__":
    print(build_library(verbose="-v" in sys.argv))
