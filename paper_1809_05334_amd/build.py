"""Build libvie.so (HIP for gfx950 + host C++) in-tree with hipcc.

Every HIP translation unit is compiled with packed-FP32 instruction
generation disabled; host-only sources are compiled by hipcc as C++.
"""
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libvie.so")
ROOT = os.path.dirname(HERE)

HIP_SOURCES = ["k_fill.hip", "k_lu.hip", "k_trsv.hip", "k_krylov.hip", "k_absorb.hip", "k_grid.hip", "api.cpp",
               "batch.cpp"]
HOST_SOURCES = ["topology.cpp", "tables.cpp", "grid.cpp"]
ARCH = os.environ.get("VIE_OFFLOAD_ARCH", "gfx950")


def hipcc():
    for c in ("/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def _run(cmd):
    p = subprocess.run(cmd, capture_output=True, text=True)
    if p.returncode != 0:
        raise RuntimeError("build failed: " + " ".join(cmd) + "\n" + p.stdout + p.stderr)
    return p.stderr


def build(verbose=False, jobs=None):
    os.makedirs(BUILD, exist_ok=True)
    cc = hipcc()
    inc = ["-I", CSRC, "-I", os.path.join(ROOT, "include")]
    common = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function", "-Wno-unused-variable"]
    cmds, objs = [], []
    for s in HIP_SOURCES:
        o = os.path.join(BUILD, s + ".o")
        cmds.append([cc, "-x", "hip", f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang",
                     "-packed-fp32-ops", "-munsafe-fp-atomics", *common, *inc, "-c", os.path.join(CSRC, s), "-o", o])
        objs.append(o)
    for s in HOST_SOURCES:
        o = os.path.join(BUILD, s + ".o")
        cmds.append([cc, "-x", "c++", *common, *inc, "-c", os.path.join(CSRC, s), "-o", o])
        objs.append(o)
    jobs = jobs or min(8, len(cmds))
    with cf.ThreadPoolExecutor(jobs) as ex:
        for err in ex.map(_run, cmds):
            if verbose and err.strip():
                sys.stderr.write(err)
    tmp = LIB + ".tmp"
    _run([cc, "-shared", f"--offload-arch={ARCH}", "-fPIC", "-o", tmp, *objs, "-L/opt/rocm/lib", "-lhipfft",
          "-Wl,-rpath,/opt/rocm/lib"])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
