"""Build the HIP library (gfx950) in-tree: paper_1309_3075_amd/libepochlik.so.

Usage: python -m paper_1309_3075_amd.build   (or build() from Python)
"""
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libepochlik.so")
BUILD_DIR = os.path.join(HERE, "_build")

HIP_SOURCES = ["epochlik.hip", "dispatch.hip", "kernels_generic.hip", "kernels_qgrad.hip", "kernels_nuc.hip", "kernels_probe.hip", "kernels_codon.hip", "kernels_pmfma.hip", "kernels_walk.hip", "kernels_eigcheck.hip", "incremental.hip", "kernels_tgrad.hip", "batch.hip"]
CPP_SOURCES = ["planner.cpp"]

ARCH = os.environ.get("EPOCHLIK_ARCH", "gfx950")
COMMON = ["-O3", "-fPIC", "-std=c++17", f"-I{CSRC}", f"-I{os.path.join(HERE, '..', 'include')}"]
# Packed FP32 instructions are kept out of every device code object.
HIP_FLAGS = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-munsafe-fp-atomics", "-ffp-contract=fast"]


def _hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError("command failed:\n" + " ".join(cmd) + "\n" + r.stdout)
    return r.stdout


def build(verbose: bool = False, jobs: int = 8) -> str:
    """Compile every HIP/C++ source for gfx950 and link libepochlik.so."""
    hipcc = _hipcc()
    os.makedirs(BUILD_DIR, exist_ok=True)
    cmds = []
    objs = []
    for src in HIP_SOURCES:
        obj = os.path.join(BUILD_DIR, src + ".o")
        cmds.append([hipcc, *COMMON, *HIP_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    for src in CPP_SOURCES:
        obj = os.path.join(BUILD_DIR, src + ".o")
        cmds.append(["g++", *COMMON, "-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        for out in ex.map(_run, cmds):
            if verbose and out:
                print(out)
    tmp = OUT + ".tmp"
    _run([hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs])
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
