"""Build the HIP/C++ library libvsr.so in-tree with hipcc for gfx950.

Usage: python -m paper_2107_14758_amd.build   (or build() from Python).
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libvsr.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

COMMON = [
    "--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17", "-fopenmp",
    # packed FP32 instructions are kept out of all device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]
SOURCES = [("kernels.hip", ["-x", "hip"]), ("transfer.hip", ["-x", "hip"]), ("patch_f32.hip", ["-x", "hip"]),
           ("patch_f64.hip", ["-x", "hip"]),
           ("surrogate.hip", ["-x", "hip"]), ("noalloc.hip", ["-x", "hip"]), ("mg.hip", ["-x", "hip"]), ("op_mfma.hip", ["-x", "hip"]), ("elastic.hip", ["-x", "hip"]), ("setup.cpp", []), ("capi.cpp", []),
           ("surrogate_capi.cpp", [])]


def _run(cmd):
    print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        sys.stdout.write(r.stdout)
        raise RuntimeError("command failed: " + " ".join(cmd))
    return r.stdout


def build(jobs=3):
    os.makedirs(BUILD, exist_ok=True)
    objs, procs = [], []
    for src, extra in SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        cmd = [HIPCC] + COMMON + extra + ["-c", os.path.join(CSRC, src), "-o", obj]
        print(" ".join(cmd), flush=True)
        procs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)))
        objs.append(obj)
    failed = None
    for cmd, p in procs:
        out, _ = p.communicate()
        if p.returncode != 0:
            sys.stdout.write(out)
            failed = cmd
    if failed:
        raise RuntimeError("compile failed: " + " ".join(failed))
    tmp = LIB + ".tmp"
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fopenmp", "-o", tmp] + objs +
         ["-Wl,-rpath,/opt/rocm/lib", "-Wl,-rpath,/opt/rocm/llvm/lib"])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
