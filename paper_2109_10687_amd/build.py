"""Build the gfx950 HIP library libddsolve.so in place (hipcc, no JIT cache).

All device code is compiled for gfx950 only.  Packed FP32 instructions are
switched off (-packed-fp32-ops) for the device pass; hipcc's host pass prints a
harmless warning that it does not know that feature.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libddsolve.so")
SOURCES = ["dd_kernels.hip", "dd_sap_fp16.hip", "dd_force.hip", "dd_mrhs.hip",
           "dd_ops.cpp", "dd_solvers.cpp", "dd_batch.cpp", "dd_capi.cpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-x", "hip",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-Xarch_host", "-fvisibility=hidden", "-I", os.path.join(HERE, "..", "include")]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    p = subprocess.run(cmd, capture_output=True, text=True)
    noise = "is not a recognized feature for this target"
    err = "\n".join(l for l in (p.stdout + p.stderr).splitlines() if noise not in l)
    if p.returncode != 0:
        raise RuntimeError(f"hipcc failed ({p.returncode}):\n{err}")
    if err.strip() and verbose:
        print(err)


def build(verbose=False, jobs=None):
    """Compile every source to an object, then link libddsolve.so."""
    from concurrent.futures import ThreadPoolExecutor
    objs = []
    cmds = []
    for src in SOURCES:
        obj = os.path.join(CSRC, os.path.splitext(src)[0] + ".o")
        objs.append(obj)
        cmds.append([HIPCC] + FLAGS + ["-c", os.path.join(CSRC, src), "-o", obj])
    with ThreadPoolExecutor(max_workers=jobs or len(cmds)) as ex:
        list(ex.map(lambda c: _run(c, verbose), cmds))
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", LIB + ".tmp"] + objs +
         ["-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx"], verbose)
    os.replace(LIB + ".tmp", LIB)
    for o in objs:
        os.remove(o)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
