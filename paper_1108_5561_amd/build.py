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
SOURCES = ["lb_device.hip", "lb_adjoint.hip", "lb_generic.hip", "lb_noalloc.hip", "lb_api.cpp", "host_setup.cpp"]

# packed FP32 instructions are disabled: the compiler would otherwise emit
# v_pk_* FP32 forms for ordinary float code
HIP_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def build(verbose=False, arch="gfx950", jobs=None):
    """Compile the sources (in parallel, `jobs` at a time) and link."""
    from concurrent.futures import ThreadPoolExecutor
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    build_dir = os.path.join(HERE, "_build")
    os.makedirs(build_dir, exist_ok=True)
    cmds, objs = [], []
    for src in SOURCES:
        obj = os.path.join(build_dir, os.path.splitext(src)[0] + ".o")
        cmd = [hipcc, "-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-result", "-Wno-unused-value",
               f"--offload-arch={arch}", "-c"]
        if src.endswith(".hip"):
            cmd += HIP_FLAGS + ["-x", "hip"]
        cmd += [os.path.join(CSRC, src), "-o", obj]
        cmds.append(cmd)
        objs.append(obj)
    if jobs is None:
        jobs = max(1, min(len(cmds), os.cpu_count() or 1, 6))

    def run(cmd):
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)

    with ThreadPoolExecutor(max_workers=jobs) as ex:
        for f in [ex.submit(run, c) for c in cmds]:
            f.result()
    tmp = OUT + ".tmp"
    cmd = [hipcc, "-shared", "-fPIC", f"--offload-arch={arch}", "-o", tmp] + objs + ["-lpthread"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
