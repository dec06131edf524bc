"""Build libcptr.so for gfx950 with hipcc (in-tree, no JIT cache).

Usage: python -m paper_1907_04229_amd.build
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libcptr.so")
OUT_HOST = os.path.join(HERE, "libcptr_host.so")
ARCH = os.environ.get("CPTR_OFFLOAD_ARCH", "gfx950")

# packed FP32 instructions are disabled (hipcc forms them from plain float
# code; some of their forms have produced wrong results on this hardware)
HIP_FLAGS = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wall", "-Wno-unused-function", "-Wno-unused-result"]
# device code: MFMA results in ordinary VGPRs (no AGPR copies); this keeps the
# learned layer kernel at 128 registers, 4 waves per SIMD
DEVICE_FLAGS = ["-mllvm", "-amdgpu-mfma-vgpr-form"]
# host setup code: no floating-point contraction, so that the aggregation
# decisions and the Galerkin entries are reproducible bit for bit
HOST_EXACT = ["-ffp-contract=off"]


def _run(cmd):
    print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd, cwd=HERE)


def build_host():
    """Host-only build of the setup algorithms (g++, no GPU code)."""
    tmp = OUT_HOST + ".tmp"
    _run(["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=off", "-Wall",
          "-o", tmp] + [os.path.join(CSRC, f) for f in
                        ("setup_amg.cpp", "setup_ilu.cpp", "setup_capi.cpp")])
    os.replace(tmp, OUT_HOST)
    return OUT_HOST


def build(verbose=True):
    hipcc = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc")
    objs = []
    for src, extra in (("setup_amg.cpp", HOST_EXACT), ("setup_ilu.cpp", HOST_EXACT),
                       ("cptr.hip", DEVICE_FLAGS)):
        obj = os.path.join(CSRC, os.path.splitext(src)[0] + ".o")
        _run([hipcc] + HIP_FLAGS + extra + ["-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    tmp = OUT + ".tmp"
    _run([hipcc, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs)
    os.replace(tmp, OUT)
    for o in objs:
        os.remove(o)
    build_host()
    return OUT


if __name__ == "__main__":
    build()
    sys.exit(0)
