"""Build the gfx950 HIP library libddsolve.so in place (hipcc, no JIT cache).

All device code is compiled for gfx950 only.  Packed FP32 instructions are
switched off (-packed-fp32-ops) for the device pass; hipcc's host pass prints a
harmless warning that it does not know that feature.

A second library, libddsolve_racecheck.so, links the same host objects with the
kernels built under -DDD_RACE_CHECK=1 (the wavefronts of every LDS-sharing
workgroup run each phase between barriers in reverse order); its results must
equal the product library's bit for bit.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libddsolve.so")
LIB_RACE = os.path.join(HERE, "libddsolve_racecheck.so")
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
    """Compile every source to an object, then link libddsolve.so and libddsolve_racecheck.so."""
    from concurrent.futures import ThreadPoolExecutor
    objs, race_objs, cmds = [], [], []
    for src in SOURCES:
        stem = os.path.join(CSRC, os.path.splitext(src)[0])
        objs.append(stem + ".o")
        cmds.append([HIPCC] + FLAGS + ["-c", os.path.join(CSRC, src), "-o", stem + ".o"])
        if src.endswith(".hip"):  # the kernels; the .cpp files hold host code only
            race_objs.append(stem + "_race.o")
            cmds.append([HIPCC] + FLAGS + ["-DDD_RACE_CHECK=1", "-c", os.path.join(CSRC, src), "-o", stem + "_race.o"])
        else:
            race_objs.append(stem + ".o")
    with ThreadPoolExecutor(max_workers=jobs or min(len(cmds), os.cpu_count() or 8)) as ex:
        list(ex.map(lambda c: _run(c, verbose), cmds))
    for lib, ob in ((LIB, objs), (LIB_RACE, race_objs)):
        _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", lib + ".tmp"] + ob +
             ["-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx"], verbose)
        os.replace(lib + ".tmp", lib)
    for o in set(objs + race_objs):
        os.remove(o)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
