"""Compile the gfx950 FDLB library (libfdlb.so) in-tree with hipcc."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libfdlb.so")
SOURCES = ["fdlb_kernels.hip", "fdlb_api.cpp", "lattice.cpp", "r1_api.cpp", "mlp_kernels.hip", "mlp_api.cpp"]
ARCH = os.environ.get("FDLB_OFFLOAD_ARCH", "gfx950")


def hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if cand and (os.path.isabs(cand) and os.path.exists(cand) or not os.path.isabs(cand)):
            return cand
    return "hipcc"


def build(verbose=False, out=None, defines=()):
    """Always recompiles; returns the path of the shared library."""
    target = out or LIB
    tmp = target + ".tmp%d" % os.getpid()
    cmd = [hipcc(), "--offload-arch=" + ARCH, "-O3", "-fPIC", "-shared", "-std=c++17",
           # keep FP32 arithmetic unpacked (no v_pk_*_f32)
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Wno-unused-command-line-argument",
           "-I", CSRC, "-I", os.path.join(os.path.dirname(HERE), "include"),
           ] + ["-D" + d for d in defines] + ["-x", "hip"] + [os.path.join(CSRC, s) for s in SOURCES] + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, target)
    return target


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
