"""Build the C-ABI shared library liblbmi.so for gfx950 with hipcc, in-tree.

Usage: python paper_1108_5561_amd/build.py   (or call build()); run as a
script, not as a module of the package, whose import loads the library.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "liblbmi.so")
SOURCES = ["lb_device.hip", "lb_adjoint.hip", "lb_noalloc.hip", "lb_api.cpp", "host_setup.cpp"]

# packed FP32 instructions are disabled: the compiler would otherwise emit
# v_pk_* FP32 forms for ordinary float code
HIP_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def build(verbose=False, arch="gfx950"):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    objs = []
    build_dir = os.path.join(HERE, "_build")
    os.makedirs(build_dir, exist_ok=True)
    for src in SOURCES:
        obj = os.path.join(build_dir, os.path.splitext(src)[0] + ".o")
        cmd = [hipcc, "-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-result", "-Wno-unused-value",
               f"--offload-arch={arch}", "-c"]
        if src.endswith(".hip"):
            cmd += HIP_FLAGS + ["-x", "hip"]
        cmd += [os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        objs.append(obj)
    tmp = OUT + ".tmp"
    cmd = [hipcc, "-shared", "-fPIC", f"--offload-arch={arch}", "-o", tmp] + objs + ["-lpthread"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
